"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/pdr.h declares, and rejects invalid instances before touching a GPU."""
import os
import re

import numpy as np
import pytest

import paper_2108_07549_amd as pdr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "pdr.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdr_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    assert set(syms) == set(pdr.EXPORTS), syms


def test_library_exports_every_declared_symbol():
    L = pdr.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def exported_definitions():
    """Body text of every exported (column-0, non-static) definition of a
    declared entry point in the library sources."""
    out = {}
    for fn in ("pdr_api.cpp", "pdr_batch.cpp", "pdr_noalloc.hip"):
        with open(os.path.join(ROOT, "paper_2108_07549_amd", "csrc", fn)) as fh:
            text = fh.read()
        for mt in re.finditer(r"^(?:pdr_status|void|const char \*)\s*(pdr_[a-z_]+)\(", text, re.M):
            start = text.index("\n{", mt.end())
            end = text.index("\n}", start)
            out[mt.group(1)] = text[start:end]
    return out


def test_every_entry_point_runs_behind_the_exception_barrier():
    """No C++ exception may cross the C ABI: every declared entry point that
    can allocate host memory wraps its body in abi_guard (or, for the destroy
    calls, a catch-all)."""
    defs = exported_definitions()
    no_alloc = {"pdr_default_options", "pdr_last_error", "pdr_batch_last_error", "pdr_tiling"}
    for name in declared_symbols():
        assert name in defs, name
        if name in no_alloc:
            continue
        body = defs[name]
        if name.endswith("destroy"):
            assert "catch (...)" in body, name
        else:
            assert "abi_guard(" in body, name


def test_default_options_are_the_papers_settings():
    o = pdr.default_options()
    assert o.method == pdr.ESO and o.precision == pdr.FP64
    a = o.agd
    assert (a.beta_init, a.beta_min, a.beta_max, a.alpha_inc, a.alpha_dec, a.inc_period) == \
        (0.25, 0.0, 0.5, 2.0, 0.5, 10)
    g = o.gdm  # Section 7.2's GDM settings; beta_min 0 selects 1/K
    assert (g.beta_init, g.beta_min, g.beta_max, g.alpha_inc, g.alpha_dec, g.inc_period,
            g.gamma) == (0.1, 0.0, 0.2, 2.0, 0.5, 10, 0.9)
    assert o.z_feasible_tol == 1e-8 and not o.stream


def _good():
    # 3 vertices, arcs 0->1, 1->2, 2->0; one commodity 0 -> 2
    return dict(n=3, row_ptr=np.array([0, 1, 2, 3]), col=np.array([1, 2, 0]),
                u=np.array([1.0, 1.0, 1.0]), s=np.array([0]), t=np.array([2]), d=np.array([0.5]))


@pytest.mark.parametrize("mutate,fragment", [
    (lambda a: a.update(n=0, row_ptr=np.array([0])), "n must be"),
    (lambda a: a.update(s=np.array([], np.int32), t=np.array([], np.int32), d=np.array([])), "K must be"),
    (lambda a: a.update(row_ptr=np.array([1, 1, 2, 3])), "row_ptr[0]"),
    (lambda a: a.update(row_ptr=np.array([0, 2, 1, 3])), "non-decreasing"),
    (lambda a: a.update(row_ptr=np.array([0, 1, 2, 2])), "row_ptr[n]"),
    (lambda a: a.update(col=np.array([1, 3, 0])), "head out of range"),
    (lambda a: a.update(col=np.array([0, 2, 0])), "self-loop"),
    (lambda a: a.update(u=np.array([1.0, -1.0, 1.0])), "capacities"),
    (lambda a: a.update(u=np.array([1.0, np.nan, 1.0])), "capacities"),
    (lambda a: a.update(u=np.array([1.0, np.inf, 1.0])), "capacities"),
    (lambda a: a.update(d=np.array([-0.5])), "demands"),
    (lambda a: a.update(d=np.array([np.nan])), "demands"),
    (lambda a: a.update(s=np.array([3])), "out of range"),
    (lambda a: a.update(t=np.array([-1])), "out of range"),
    (lambda a: a.update(t=np.array([0])), "s_k == t_k"),
])
def test_init_rejects_invalid_instances(mutate, fragment):
    a = _good()
    mutate(a)
    with pytest.raises(pdr.PdrError) as ei:
        pdr.Context(a["n"], a["row_ptr"], a["col"], a["u"], a["s"], a["t"], a["d"])
    assert ei.value.status == 1 and fragment in ei.value.message
    assert fragment in pdr.lib().pdr_last_error(None).decode()


def test_init_rejects_isolated_commodity_endpoint():
    # vertex 3 has no arcs: its height (Delta / degree) is undefined
    with pytest.raises(pdr.PdrError) as ei:
        pdr.Context(4, np.array([0, 1, 2, 3, 3]), np.array([1, 2, 0]), np.ones(3),
                    np.array([0]), np.array([3]), np.array([1.0]))
    assert ei.value.status == 1 and "degree 0" in ei.value.message


@pytest.mark.parametrize("opts,fragment", [
    (dict(method=7), "unknown method"),
    (dict(precision=3), "unknown precision"),
    (dict(method=pdr.AGD, agd=dict(beta_init=0.0)), "AGD parameters"),
    (dict(method=pdr.AGD, agd=dict(alpha_dec=float("nan"))), "AGD parameters"),
    (dict(method=pdr.GDM, agd=dict(beta_max=0.0)), "GDM parameters"),
    (dict(method=pdr.GDM, agd=dict(gamma=1.0)), "gamma"),
    (dict(method=pdr.GDM, agd=dict(gamma=-0.1)), "gamma"),
    (dict(z_feasible_tol=-1.0), "z_feasible_tol"),
    (dict(lanes_per_arc=3), "tiling"),
    (dict(lanes_per_arc=1, vec_per_lane=1), "tiling"),  # K=100 needs more than 1 x 1 vectors
    (dict(cache_policy=3), "cache_policy"),
    (dict(cache_policy=-1), "cache_policy"),
    (dict(height_kernel=3), "height_kernel"),
    (dict(height_kernel=-1), "height_kernel"),
    (dict(height_chunk=48), "height_chunk"),
    (dict(height_chunk=131072), "height_chunk"),
])
def test_init_rejects_invalid_options(opts, fragment):
    a = _good()
    s = np.zeros(100, np.int32)
    t = np.full(100, 2, np.int32)
    with pytest.raises(pdr.PdrError) as ei:
        pdr.Context(a["n"], a["row_ptr"], a["col"], a["u"], s, t, np.ones(100), **opts)
    assert ei.value.status == 1 and fragment in ei.value.message


def test_requested_tiling_that_misses_the_row_is_rejected():
    """A requested register-resident tiling shorter than the row is refused
    before any device call (rows that long take the automatic streamed tiling)."""
    a = _good()
    K = 40000  # FP64 rows above 1024 lanes x 8 vectors x 2 values
    with pytest.raises(pdr.PdrError) as ei:
        pdr.Context(a["n"], a["row_ptr"], a["col"], a["u"], np.zeros(K, np.int32),
                    np.full(K, 2, np.int32), np.ones(K), lanes_per_arc=1024, vec_per_lane=8)
    assert ei.value.status == 1 and "tiling" in ei.value.message


def test_null_context_calls_are_invalid():
    L = pdr.lib()
    assert L.pdr_sweep(None, 1, 0.0, 0.0) == 1
    assert L.pdr_flows(None, None) == 1
    assert L.pdr_residual(None, None) == 1
    L.pdr_destroy(None)  # ignored


def test_batch_init_rejects_empty_input():
    """Checked before any device call."""
    import ctypes as C
    L = pdr.lib()
    h = C.c_void_p()
    arr = (pdr.Instance * 1)()
    assert L.pdr_batch_init(C.byref(h), 0, arr, None) == 1
    assert "B >= 1" in L.pdr_batch_last_error(None).decode()
    assert L.pdr_batch_init(C.byref(h), 2, None, None) == 1
    assert not h.value


def test_batch_and_adjoint_null_handles_are_invalid():
    import ctypes as C
    L = pdr.lib()
    assert L.pdr_batch_sweep(None, 1, 0.0, 0.0) == 1
    assert L.pdr_batch_tune(None, 1, None) == 1
    assert L.pdr_batch_stopped(None, None) == 1
    z = C.c_double()
    assert L.pdr_adjoint(None, 1, 0, C.byref(z), None, None) == 1
    L.pdr_batch_destroy(None)  # ignored


def test_autograd_function_checks_dtypes_before_any_call():
    """The torch.autograd.Function over pdr_adjoint takes float64 u and d and
    refuses others before it reaches the library."""
    torch = pytest.importorskip("torch")
    from gen.instance import recipe_grid4_k8
    from paper_2108_07549_amd.autograd import residual_after_sweeps
    inst = recipe_grid4_k8()
    with pytest.raises(TypeError):
        residual_after_sweeps(inst, torch.tensor(inst.u, dtype=torch.float32),
                              torch.tensor(inst.d, dtype=torch.float64), 4)


def test_flows_device_checks_the_tensor_before_any_call():
    """A tensor the library would write past, or read as the wrong type, is
    refused by the binding before any library call."""
    import ctypes
    import torch
    c = pdr.Context.__new__(pdr.Context)
    c._h, c._keep = ctypes.c_void_p(), None
    c.n, c.m, c.K = 4, 6, 3
    for t, fp64 in ((torch.empty(18, dtype=torch.float64), True),
                    (torch.empty(18, dtype=torch.float32), False)):
        with pytest.raises(ValueError):
            c.flows_device(t, fp64)


HOST_OOM = r"""
import ctypes as C, resource, sys
import numpy as np
sys.path.insert(0, {root!r})
import paper_2108_07549_amd as pdr
L = pdr.lib()
n = 50_000_000  # init's first host arrays then need 200 MB
rp = np.zeros(n + 1, np.int64)
one = np.zeros(1, np.int32)
s, t, ud = np.array([0], np.int32), np.array([1], np.int32), np.ones(1)
vm = [int(x.split()[1]) for x in open("/proc/self/status") if x.startswith("VmSize")][0] * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (64 << 20), resource.RLIM_INFINITY))
h = C.c_void_p()
p = lambda a: a.ctypes.data_as(C.c_void_p)
st = L.pdr_init(C.byref(h), n, 0, p(rp), p(one), p(ud), 1, p(s), p(t), p(ud), None)
print(st, h.value is None, L.pdr_last_error(None).decode())
"""


def test_host_allocation_failure_is_a_status_not_an_exception():
    """Under an address-space limit, pdr_init's host arrays cannot be allocated:
    the call returns PDR_ERR_OOM with its text (a C++ exception crossing the C
    ABI would abort the process). Runs in a child process with the limit set
    after the library is loaded; init fails before any device call."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", HOST_OOM.format(root=ROOT)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    st, null_handle, msg = r.stdout.strip().split(" ", 2)
    assert int(st) == 2 and null_handle == "True"
    assert "host memory allocation failed" in msg


C_CALLER = r"""
#include <stdio.h>
#include <string.h>
#include "pdr.h"

int main(void)
{
    pdr_options o;
    pdr_default_options(&o);
    if (o.method != PDR_ESO || o.precision != PDR_FP64 || o.agd.beta_init != 0.25 ||
        o.gdm.gamma != 0.9 || o.z_feasible_tol != 1e-8 || o.stream != NULL)
        return 10;
    /* a triangle 0 -> 1 -> 2 -> 0 with a self-loop 2 -> 2 appended: rejected
       before any device call */
    const int64_t row_ptr[4] = {0, 1, 2, 4};
    const int32_t col[4] = {1, 2, 0, 2};
    const double u[4] = {1, 1, 1, 1};
    const int32_t s[1] = {0}, t[1] = {2};
    const double d[1] = {1};
    pdr_ctx *ctx = (pdr_ctx *)1;
    pdr_status st = pdr_init(&ctx, 3, 4, row_ptr, col, u, 1, s, t, d, &o);
    if (st != PDR_ERR_INVALID || ctx != NULL) return 11;
    const char *msg = pdr_last_error(NULL);
    if (msg == NULL || strstr(msg, "self-loop") == NULL) return 12;
    if (pdr_sweep(NULL, 1, 0.0, 0.0) != PDR_ERR_INVALID) return 13;
    pdr_destroy(NULL);
    printf("ok\n");
    return 0;
}
"""


def test_header_is_plain_c_and_the_library_serves_a_c_caller(tmp_path):
    """include/pdr.h compiles as strict C99 (-pedantic -Werror), and a C program
    linked against libpdr.so gets the defaults of the paper's settings and the
    documented argument errors, with no Python in between."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "caller.c"
    src.write_text(C_CALLER)
    exe = tmp_path / "caller"
    libdir = os.path.dirname(pdr.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", libdir, "-lpdr", "-Wl,-rpath," + libdir])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stderr[-2000:])
