"""The library driven from C alone (no Python between the caller and the ABI):
a C program compiled against include/pdr.h and linked to libpdr.so runs PDR-ESO
passes on the GPU and reads back flows and the residual report, checked
against the closed forms of the two-vertex example."""
import os
import shutil
import subprocess
import sys

import pytest

import paper_2108_07549_amd as pdr

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <math.h>
#include <stdio.h>
#include "pdr.h"

#define CHECK(x) do { pdr_status st_ = (x); if (st_ != PDR_OK) { \
    fprintf(stderr, "%s -> %d: %s\n", #x, (int)st_, pdr_last_error(ctx)); return 20; } } while (0)

int main(void)
{
    /* vertices 0 and 1, arcs 0 -> 1 and 1 -> 0 of capacity 8; one commodity
       0 -> 1 of demand 10 > 8: infeasible */
    const int64_t row_ptr[3] = {0, 1, 2};
    const int32_t col[2] = {1, 0};
    const double u[2] = {8, 8};
    const int32_t s[1] = {0}, t[1] = {1};
    const double d[1] = {10};
    pdr_ctx *ctx = NULL;
    pdr_options o;
    pdr_default_options(&o);
    if (pdr_init(&ctx, 2, 2, row_ptr, col, u, 1, s, t, d, &o) != PDR_OK) {
        fprintf(stderr, "init: %s\n", pdr_last_error(NULL));
        return 10;
    }
    double f[2];
    CHECK(pdr_sweep(ctx, 6, 0.0, 0.0));
    CHECK(pdr_flows(ctx, f));
    printf("f6 %.17g %.17g\n", f[0], f[1]);
    CHECK(pdr_sweep(ctx, 200, 0.0, 0.0));
    pdr_residual_t r;
    CHECK(pdr_residual(ctx, &r));
    CHECK(pdr_flows(ctx, f));
    printf("f %.17g %.17g\n", f[0], f[1]);
    printf("z %.17g gap %.17g verdict %d sweeps %lld\n", r.z, r.farkas_gap, (int)r.verdict,
           (long long)r.sweeps_done);
    pdr_destroy(ctx);
    return 0;
}
"""


def test_c_program_runs_passes_and_reads_results(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "two_vertex.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "two_vertex"
    libdir = os.path.dirname(pdr.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe), "-L", libdir, "-lpdr", "-Wl,-rpath," + libdir,
                           "-lm"])
    print("[gpu-c] running the C caller", flush=True)
    sys.stdout.flush()
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    out = {}
    for line in r.stdout.splitlines():
        p = line.split()
        out[p[0]] = p[1:]
    print("[gpu-c]", out, flush=True)
    # ESO from f = 0: f_1 = (d + f)/2 while uncongested, then (d + f + u)/3; the
    # sixth pass gives 485/54, the limit (d + u)/2 = 9 with z* = 1 and G = 2 z*
    assert float(out["f6"][0]) == pytest.approx(485 / 54, abs=1e-12) and float(out["f6"][1]) == 0.0
    assert float(out["f"][0]) == pytest.approx(9.0, abs=1e-12) and float(out["f"][1]) == 0.0
    assert float(out["z"][0]) == pytest.approx(1.0, abs=1e-12)
    assert float(out["z"][2]) == pytest.approx(2.0, abs=1e-12)
    assert int(out["z"][4]) == 2  # PDR_INFEASIBLE
    assert int(out["z"][6]) == 206
