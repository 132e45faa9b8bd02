// Host side of the C ABI declared in include/pdr.h: argument validation,
// device memory, the stream, and the launch sequence of a sweep.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <limits>
#include <string>
#include <vector>

#include "pdr.h"
#include "pdr_context.h"
#include "pdr_internal.h"

using namespace pdr_host;
using pdr::Ctrl;
using pdr::DevGraph;
using pdr::Tiling;

namespace pdr_host {
thread_local std::string g_init_error;

int pow2ceil(int64_t x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

void *cur_f(pdr_ctx *c) { return c->precision == PDR_FP64 ? (void *)c->f64 : (void *)c->f32; }

void *cur_v(pdr_ctx *c) { return c->precision == PDR_FP64 ? (void *)c->v64 : (void *)c->v32; }

void *cur_h(pdr_ctx *c) { return c->precision == PDR_FP64 ? (void *)c->h64 : (void *)c->h32; }

pdr::AgdParams agd_params(const pdr_ctx *c)
{
    return pdr::AgdParams{c->beta_min, c->agd.beta_max, c->agd.alpha_inc, c->agd.alpha_dec,
                          c->agd.inc_period, c->agd.gamma};
}
}  // namespace pdr_host

// ------------------------------------------------------------------ helpers
namespace {

pdr_status fail(pdr_ctx *c, pdr_status st, const std::string &msg)
{
    c->err = msg;
    return st;
}

pdr_status dev_fail(pdr_ctx *c, hipError_t e, const char *what)
{
    c->poisoned = true;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return PDR_ERR_DEVICE;
}

#define PDR_CHECK(ctx, expr)                                          \
    do {                                                              \
        hipError_t _e = (expr);                                       \
        if (_e != hipSuccess) return dev_fail((ctx), _e, #expr);      \
    } while (0)

template <typename T>
hipError_t dalloc(pdr_ctx *c, T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    c->allocs.push_back(nullptr);  // the slot first, so a failed push leaks nothing
    hipError_t e = hipMalloc(&c->allocs.back(), count * sizeof(T));
    if (e == hipSuccess)
        *p = static_cast<T *>(c->allocs.back());
    else
        c->allocs.pop_back();
    return e;
}

template <typename T>
hipError_t upload(pdr_ctx *c, T **p, const T *src, size_t count)
{
    hipError_t e = dalloc(c, p, count);
    if (e != hipSuccess) return e;
    if (count) e = hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}



int vec_of(int32_t precision) { return precision == PDR_FP64 ? 2 : 4; }

// Fewest register vectors per lane (a supported count) that cover nvec with L lanes;
// 0 if none does.
int cover_nv(int64_t nvec, int L)
{
    const int need = (int)((nvec + L - 1) / L);
    for (int cand = need < 1 ? 1 : need; cand <= kMaxNv; ++cand)
        if (pdr::tiling_supported(L, cand)) return cand;
    return 0;
}

Tiling auto_tiling(int32_t Kp, int32_t precision, int32_t method)
{
    const int64_t nvec = Kp / vec_of(precision);
    // rows longer than any register-resident tiling holds are streamed
    if (nvec > pdr::max_tiling_vectors()) return pdr::streamed_tiling();
    // about five register vectors per lane: long rows get many lanes, and
    // the blocks stay small enough that several arcs share a CU
    int L = pow2ceil((nvec + 4) / 5);
    if (L > kMaxLanes) L = kMaxLanes;
    // the gradient steps reduce once per arc (no threshold passes): they run
    // best with at most 512 lanes and more vectors per lane
    if ((method == PDR_AGD || method == PDR_GDM) && L > 512 && cover_nv(nvec, 512) > 0) L = 512;
    int nv = cover_nv(nvec, L);
    if (nv < 1) nv = pow2ceil((nvec + L - 1) / L);
    return Tiling{L, nv};
}

bool tiling_covers(Tiling tl, int32_t Kp, int32_t precision)
{
    const int64_t nvec = Kp / vec_of(precision);
    if (tl.nv < 0) return pdr::tiling_supported(tl.lanes, tl.nv);  // streamed: any length
    return pdr::tiling_supported(tl.lanes, tl.nv) && (int64_t)tl.lanes * tl.nv >= nvec;
}

pdr_status choose_tiling(pdr_ctx *c, int32_t precision, Tiling *out)
{
    Tiling tl = auto_tiling(c->Kp, precision, c->method);
    if (c->req_lanes > 0 || c->req_nv > 0) {
        tl.lanes = c->req_lanes > 0 ? c->req_lanes : tl.lanes;
        tl.nv = c->req_nv > 0 ? c->req_nv : pow2ceil((c->Kp / vec_of(precision) + tl.lanes - 1) /
                                                    tl.lanes);
    }
    if (!tiling_covers(tl, c->Kp, precision)) {
        char buf[400];
        const int mv = pdr::max_tiling_vectors();
        snprintf(buf, sizeof buf,
                 "the requested arc tiling (lanes %d x vectors %d) does not cover K=%d "
                 "(padded %d) in this precision (a register-resident row holds at most %d "
                 "vectors of 16 bytes: %d commodities in FP64, %d in FP32 bulk; longer rows "
                 "take the automatic streamed tiling)",
                 tl.lanes, tl.nv, c->K, c->Kp, mv, 2 * mv, 4 * mv);
        c->err = buf;
        return PDR_ERR_INVALID;
    }
    *out = tl;
    return PDR_OK;
}

bool usable(pdr_ctx *c, pdr_status *st)
{
    if (!c) {
        *st = PDR_ERR_INVALID;
        return false;
    }
    if (c->poisoned) {
        *st = PDR_ERR_DEVICE;
        return false;
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) {
        *st = dev_fail(c, e, "hipSetDevice");
        return false;
    }
    return true;
}

// Vectors per commodity chunk of the height kernel: a whole 256-thread block
// per (vertex, chunk) when rows are long, several vertices per block otherwise.
void set_height_chunk(pdr_ctx *c)
{
    const int64_t nvec = c->Kp / vec_of(c->precision);
    const int cap = c->req_height_chunk > 0 ? c->req_height_chunk : kHeightChunkAuto;
    c->g.height_cv = std::min<int>(cap, pow2ceil(nvec));
    // A small instance leaves few height items per thread and the kernel is
    // latency-bound: in FP64 one batch of 8 rows then covers most vertices'
    // incidence lists; in FP32 (half the items) twice the resident grid lets
    // the dispatcher even out the last round of items.
    const int64_t items = (int64_t)c->n * nvec;
    int grid = kHeightGridAuto, unroll = kHeightUnrollAuto;
    if (c->precision == PDR_FP64 && items < 16 * 256 * (int64_t)kHeightGridAuto) unroll = 8;
    if (c->precision != PDR_FP64 && items < 4 * 256 * (int64_t)kHeightGridAuto)
        grid = 2 * kHeightGridAuto;
    c->g.height_grid = c->req_height_grid > 0 ? c->req_height_grid : grid;
    c->g.height_unroll = c->req_height_unroll > 0 ? c->req_height_unroll : unroll;
    c->g.tile_grid = c->req_height_grid > 0 ? c->req_height_grid : kTileGridAuto;
}





pdr_status ensure_buffers(pdr_ctx *c, int32_t precision)
{
    const size_t mK = (size_t)c->m * c->Kp, nK = (size_t)c->n * c->Kp;
    if (precision == PDR_FP64) {
        if (!c->f64) {
            hipError_t e = dalloc(c, &c->f64, mK);
            if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (f)");
            PDR_CHECK(c, e);
        }
    } else {
        if (!c->f32) {
            hipError_t e = dalloc(c, &c->f32, mK);
            if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (f)");
            PDR_CHECK(c, e);
        }
        if (!c->h32) {
            hipError_t e = dalloc(c, &c->h32, nK);
            if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (h)");
            PDR_CHECK(c, e);
        }
    }
    if (c->method == PDR_GDM) {  // velocities of Algorithm 4, in the storage precision
        hipError_t e = precision == PDR_FP64 ? (c->v64 ? hipSuccess : dalloc(c, &c->v64, mK))
                                             : (c->v32 ? hipSuccess : dalloc(c, &c->v32, mK));
        if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (v)");
        PDR_CHECK(c, e);
    }
    if (!c->h64) {  // FP64 heights: the FP64 sweep's h and every residual report
        hipError_t e = dalloc(c, &c->h64, nK);
        if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (h)");
        PDR_CHECK(c, e);
    }
    // undo rows of the streamed AGD / GDM kernels, sized for FP64 rows so they
    // serve either precision; needed when FP64 rows are streamed (or a
    // streamed tiling was asked for)
    const bool agd_like = c->method == PDR_AGD || c->method == PDR_GDM;
    if (agd_like && !c->d_undo && (c->Kp / 2 > pdr::max_tiling_vectors() || c->req_nv < 0)) {
        const size_t rows = (size_t)pdr::kStreamSlots * (c->method == PDR_GDM ? 2 : 1);
        hipError_t e = dalloc(c, &c->d_undo, rows * (size_t)c->Kp);
        if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (undo rows)");
        PDR_CHECK(c, e);
    }
    c->g.stream_undo = c->d_undo;
    return PDR_OK;
}

pdr_status sync_ctrl(pdr_ctx *c)
{
    PDR_CHECK(c, hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}

pdr_status push_ctrl(pdr_ctx *c)
{
    PDR_CHECK(c, hipMemcpyAsync(c->ctrl, c->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}

// Processing order with locality: vertices are grouped into clusters of up to
// T vertices grown by breadth-first search over the undirected adjacency, the
// cluster seeds taken in a breadth-first order of the whole graph, so that
// neighbouring clusters follow each other. The kernels visit vertices
// (height) and out-arcs (arc update) in this order, so the rows of f and h
// that several vertices or arcs share are read close together in time. Only
// the visiting order changes; the data layout and every result are the same.
// cstart receives the first position of each cluster and then n (one
// cluster, {0, n}, for the caller's order).
void locality_order(int32_t n, const int32_t *rp, const int32_t *col,
                    const std::vector<int32_t> &in_ptr, const std::vector<int32_t> &in_idx,
                    const std::vector<int32_t> &tails, int32_t T, std::vector<int32_t> &vorder,
                    std::vector<int32_t> &aorder, std::vector<int32_t> &cstart)
{
    vorder.clear();
    aorder.clear();
    cstart.clear();
    if (T <= 1) {
        for (int32_t v = 0; v < n; ++v) vorder.push_back(v);
        cstart.push_back(0);
    } else {
        std::vector<char> seen(n, 0), taken(n, 0);
        std::vector<int32_t> seeds, queue;
        seeds.reserve(n);
        // global breadth-first order (over every component)
        for (int32_t r = 0; r < n; ++r) {
            if (seen[r]) continue;
            size_t head = seeds.size();
            seeds.push_back(r);
            seen[r] = 1;
            while (head < seeds.size()) {
                const int32_t v = seeds[head++];
                auto visit = [&](int32_t w) {
                    if (!seen[w]) {
                        seen[w] = 1;
                        seeds.push_back(w);
                    }
                };
                for (int32_t e = rp[v]; e < rp[v + 1]; ++e) visit(col[e]);
                for (int32_t p = in_ptr[v]; p < in_ptr[v + 1]; ++p) visit(tails[in_idx[p]]);
            }
        }
        std::vector<int32_t> stamp(n, -1);
        int32_t cl = 0;
        for (int32_t sd : seeds) {
            if (taken[sd]) continue;
            cstart.push_back((int32_t)vorder.size());
            queue.clear();
            queue.push_back(sd);
            stamp[sd] = cl;
            size_t head = 0;
            int32_t size = 0;
            while (head < queue.size() && size < T) {
                const int32_t v = queue[head++];
                if (taken[v]) continue;
                taken[v] = 1;
                vorder.push_back(v);
                ++size;
                auto visit = [&](int32_t w) {
                    if (!taken[w] && stamp[w] != cl) {
                        stamp[w] = cl;
                        queue.push_back(w);
                    }
                };
                for (int32_t e = rp[v]; e < rp[v + 1]; ++e) visit(col[e]);
                for (int32_t p = in_ptr[v]; p < in_ptr[v + 1]; ++p) visit(tails[in_idx[p]]);
            }
            ++cl;
        }
    }
    cstart.push_back(n);
    for (int32_t v : vorder)
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) aorder.push_back(e);
}

// Tiles of the tiled height kernel: runs of consecutive visiting positions
// within one locality cluster, each closed before it would hold more than
// kTileVerts vertices or kTileArcs distinct incident arcs. tinfo gets (first
// position, end position, first slot, end slot) per tile, tarc the tile's
// arcs in order of first incidence, tslot[p] the slot of vinc[p] in its
// tile. Returns false when one vertex alone has more than kTileArcs incident
// arcs (the vertex-parallel kernel then runs).
bool build_tiles(int32_t m, const std::vector<int32_t> &vinfo, const std::vector<int32_t> &vinc,
                 const std::vector<int32_t> &cstart, int32_t max_verts, int32_t max_arcs,
                 std::vector<int32_t> &tinfo, std::vector<int32_t> &tarc,
                 std::vector<uint16_t> &tslot)
{
    tinfo.clear();
    tarc.clear();
    tslot.assign(vinc.size(), 0);
    std::vector<int32_t> mark((size_t)m, -1), slot_of((size_t)m, 0);
    int32_t tiles = 0;
    for (size_t ci = 0; ci + 1 < cstart.size(); ++ci) {
        int32_t pos = cstart[ci];
        const int32_t end = cstart[ci + 1];
        while (pos < end) {
            const int32_t first = pos, a0 = (int32_t)tarc.size();
            int32_t na = 0;
            while (pos < end && pos - first < max_verts) {
                const int32_t p0 = vinfo[8 * (size_t)pos + 1], p1 = vinfo[8 * (size_t)pos + 3];
                int32_t add = 0;
                for (int32_t p = p0; p < p1; ++p) add += mark[vinc[p]] != tiles;
                if (na + add > max_arcs) break;
                for (int32_t p = p0; p < p1; ++p) {
                    const int32_t e = vinc[p];
                    if (mark[e] != tiles) {
                        mark[e] = tiles;
                        slot_of[e] = na++;
                        tarc.push_back(e);
                    }
                    tslot[p] = (uint16_t)slot_of[e];
                }
                ++pos;
            }
            if (pos == first) return false;
            tinfo.insert(tinfo.end(), {first, pos, a0, a0 + na});
            ++tiles;
        }
    }
    return true;
}



// Enqueue `count` passes (height, objective + stop test, arc update) on st.
hipError_t enqueue_passes(pdr_ctx *c, int64_t count, hipStream_t st)
{
    const bool fp64 = c->precision == PDR_FP64;
    void *f = cur_f(c);
    void *h = cur_h(c);
    const pdr::AgdParams prm = agd_params(c);
    for (int64_t q = 0; q < count; ++q) {
        hipError_t e = pdr::launch_height(c->g, fp64, f, h, c->zpart, c->Fsum, c->ctrl, c->zlog,
                                          c->zlog_cap - 1, st);
        if (e == hipSuccess)
            e = c->method == PDR_ESO || c->method == PDR_CAP
                    ? pdr::launch_eso(c->g, fp64, c->tiling, f, h, c->Fsum, c->ctrl,
                                      c->method == PDR_CAP, st)
                    : pdr::launch_agd(c->g, fp64, c->tiling, f, h, c->Fsum, c->beta, prm, c->ctrl,
                                      c->method == PDR_GDM ? cur_v(c) : nullptr, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The graph of graph_sweeps passes for the current precision (kernels only;
// the kernels read the stop flag, so passes after a stop do nothing).
pdr_status sweep_graph(pdr_ctx *c, hipGraphExec_t *out)
{
    hipGraphExec_t &ge = c->gexec[c->precision];
    if (!ge) {
        if (!c->cap_stream) PDR_CHECK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        PDR_CHECK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_passes(c, c->graph_sweeps, c->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
        PDR_CHECK(c, e);
        PDR_CHECK(c, e2);
        e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        PDR_CHECK(c, e);
    }
    *out = ge;
    return PDR_OK;
}

void free_all(pdr_ctx *c)
{
    // teardown: failures here cannot be reported and leave nothing to undo
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    if (c->h_res) (void)hipHostFree(c->h_res);
    c->h_ctrl = nullptr;
    c->h_res = nullptr;
    for (auto &ge : c->gexec)
        if (ge) (void)hipGraphExecDestroy(ge);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

void pdr_default_options(pdr_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->method = PDR_ESO;
    opt->precision = PDR_FP64;
    opt->agd.beta_init = 0.25;
    opt->agd.beta_min = 0.0;  // 1/K
    opt->agd.beta_max = 0.5;
    opt->agd.alpha_inc = 2.0;
    opt->agd.alpha_dec = 0.5;
    opt->agd.inc_period = 10;
    opt->agd.gamma = 0.0;
    opt->gdm.beta_init = 0.1;
    opt->gdm.beta_min = 0.0;  // 1/K
    opt->gdm.beta_max = 0.2;
    opt->gdm.alpha_inc = 2.0;
    opt->gdm.alpha_dec = 0.5;
    opt->gdm.inc_period = 10;
    opt->gdm.gamma = 0.9;
    opt->z_feasible_tol = 1e-8;
    opt->stream = nullptr;
    opt->lanes_per_arc = 0;
    opt->vec_per_lane = 0;
    opt->graph_sweeps = 0;
    opt->height_chunk = 0;
    opt->cluster_size = 0;
    opt->height_blocks = 0;
    opt->height_unroll = 0;
    opt->z_log_capacity = 0;
    opt->cache_policy = 0;
    opt->batch_groups = 0;
    opt->height_kernel = 0;
}

const char *pdr_last_error(const pdr_ctx *ctx)
{
    if (!ctx) return g_init_error.c_str();
    return ctx->err.c_str();
}

static pdr_status init_fail(pdr_ctx *c, pdr_status st, pdr_ctx **out)
{
    g_init_error = c->err;
    free_all(c);
    delete c;
    *out = nullptr;
    return st;
}

// *created receives the context as soon as it exists, so that the exception
// barrier of pdr_init can free it if the body is left part way.
static pdr_status pdr_init_body(pdr_ctx **out, int32_t n, int32_t m, const int64_t *row_ptr,
                                const int32_t *col, const double *u, int32_t K,
                                const int32_t *s, const int32_t *t, const double *d,
                                const pdr_options *opt_in, pdr_ctx **created)
{
    if (!out) {
        g_init_error = "out is NULL";
        return PDR_ERR_INVALID;
    }
    *out = nullptr;
    pdr_options opt;
    pdr_default_options(&opt);
    if (opt_in) opt = *opt_in;
    auto invalid = [&](const std::string &msg) {
        g_init_error = msg;
        return PDR_ERR_INVALID;
    };
    // ---- instance validation (Section 1: G(V, E), u: E -> Q+, (s_k, t_k, d_k), s_k != t_k)
    if (n < 1) return invalid("n must be >= 1");
    if (m < 0) return invalid("m must be >= 0");
    if (K < 1) return invalid("K must be >= 1");
    if (!row_ptr || (m > 0 && (!col || !u)) || !s || !t || !d)
        return invalid("a required array is NULL");
    if (row_ptr[0] != 0) return invalid("row_ptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return invalid("row_ptr must be non-decreasing");
    if (row_ptr[n] != (int64_t)m) return invalid("row_ptr[n] must equal m");
    std::vector<int32_t> deg(n, 0), tails(m);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n) return invalid("arc head out of range");
            if (col[e] == i) return invalid("self-loop arcs are not allowed");
            tails[e] = i;
            deg[i] += 1;
            deg[col[e]] += 1;
        }
    for (int32_t e = 0; e < m; ++e)
        if (!finite_nonneg(u[e])) return invalid("capacities must be finite and >= 0");
    for (int32_t k = 0; k < K; ++k) {
        if (s[k] < 0 || s[k] >= n || t[k] < 0 || t[k] >= n)
            return invalid("commodity endpoint out of range");
        if (s[k] == t[k]) return invalid("commodity with s_k == t_k");
        if (!finite_nonneg(d[k])) return invalid("demands must be finite and >= 0");
        if (deg[s[k]] == 0 || deg[t[k]] == 0)
            return invalid("commodity endpoint has degree 0 (its height is undefined)");
    }
    // ---- options
    if (opt.method != PDR_ESO && opt.method != PDR_AGD && opt.method != PDR_GDM &&
        opt.method != PDR_CAP)
        return invalid("unknown method");
    if (opt.precision != PDR_FP64 && opt.precision != PDR_FP32_BULK)
        return invalid("unknown precision");
    if (opt.method == PDR_AGD || opt.method == PDR_GDM) {
        const pdr_agd_params &a = opt.method == PDR_AGD ? opt.agd : opt.gdm;
        if (!(a.beta_init > 0) || !(a.beta_max > 0) || !(a.alpha_inc > 0) || !(a.alpha_dec > 0) ||
            !std::isfinite(a.beta_init) || !std::isfinite(a.beta_max) ||
            !std::isfinite(a.alpha_inc) || !std::isfinite(a.alpha_dec) ||
            !std::isfinite(a.beta_min) || a.inc_period < 0)
            return invalid(opt.method == PDR_AGD ? "invalid AGD parameters" : "invalid GDM parameters");
        if (opt.method == PDR_GDM && !(a.gamma >= 0.0 && a.gamma < 1.0))
            return invalid("GDM momentum gamma must lie in [0, 1)");
    }
    if (!(opt.z_feasible_tol >= 0) || !std::isfinite(opt.z_feasible_tol))
        return invalid("z_feasible_tol must be finite and >= 0");
    if (opt.lanes_per_arc < 0 || opt.vec_per_lane < 0) return invalid("negative tiling request");
    if (opt.cluster_size < 0) return invalid("cluster_size must be >= 0");
    if (opt.height_unroll != 0 && opt.height_unroll != 1 && opt.height_unroll != 2 &&
        opt.height_unroll != 4 && opt.height_unroll != 8)
        return invalid("height_unroll must be 0, 1, 2, 4 or 8");
    if (opt.z_log_capacity < 0 || opt.z_log_capacity > pdr::kZLogCap ||
        (opt.z_log_capacity & (opt.z_log_capacity - 1)) != 0)
        return invalid("z_log_capacity must be 0 or a power of two up to 2^20");
    if (opt.cache_policy < 0 || opt.cache_policy > 2)
        return invalid("cache_policy must be 0, 1 or 2");
    if (opt.height_blocks < 0 || opt.height_blocks > pdr::kHeightBlocksMax)
        return invalid("height_blocks must be 0 or 1..8192");
    if (opt.height_kernel < 0 || opt.height_kernel > 2)
        return invalid("height_kernel must be 0, 1 or 2");
    if (opt.height_chunk < 0 || opt.height_chunk > 65536 ||
        (opt.height_chunk & (opt.height_chunk - 1)) != 0)
        return invalid("height_chunk must be 0 or a power of two up to 65536");

    pdr_ctx *c = new pdr_ctx();
    *created = c;
    c->n = n;
    c->m = m;
    c->K = K;
    c->Kp = (int32_t)(K <= 64 ? (K + 3) / 4 * 4 : (K + 31) / 32 * 32);
    c->method = opt.method;
    c->precision = opt.precision;
    c->agd = opt.method == PDR_GDM ? opt.gdm : opt.agd;
    if (opt.method != PDR_GDM) c->agd.gamma = 0.0;
    c->beta_min = c->agd.beta_min > 0 ? c->agd.beta_min : 1.0 / K;
    c->z_feasible_tol = opt.z_feasible_tol;
    c->req_lanes = opt.lanes_per_arc;
    c->req_nv = opt.vec_per_lane;
    c->graph_sweeps = opt.graph_sweeps == 0 ? 32 : (opt.graph_sweeps < 0 ? 0 : opt.graph_sweeps);
    c->req_height_chunk = opt.height_chunk;
    c->cluster_size = opt.cluster_size == 0 ? kClusterAuto : opt.cluster_size;
    c->req_height_grid = opt.height_blocks;
    c->req_height_unroll = opt.height_unroll;
    c->req_cache_policy = opt.cache_policy;
    c->req_height_kernel = opt.height_kernel;
    if (opt.z_log_capacity > 0) c->zlog_cap = opt.z_log_capacity;
    {
        pdr_status st = choose_tiling(c, c->precision, &c->tiling);
        if (st != PDR_OK) return init_fail(c, st, out);
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        c->err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return init_fail(c, PDR_ERR_DEVICE, out);
    }
    {
        // the staging array of pdr_set_state_noalloc: its device address, once per device
        double *scratch = nullptr;
        e = noalloc_scratch(c->device, &scratch, nullptr);
        if (e != hipSuccess) {
            c->err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
            return init_fail(c, PDR_ERR_DEVICE, out);
        }
    }
    if (opt.stream) {
        c->stream = (hipStream_t)opt.stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            c->err = std::string("hipStreamCreate: ") + hipGetErrorString(e);
            return init_fail(c, PDR_ERR_DEVICE, out);
        }
        c->own_stream = true;
    }

    // ---- memory estimate before any allocation
    {
        const double w = c->precision == PDR_FP64 ? 8.0 : 4.0;
        const double mK = (double)m * c->Kp, nK = (double)n * c->Kp;
        double need = mK * w * (opt.method == PDR_GDM ? 2.0 : 1.0) + nK * w + nK * 8.0 * (c->precision == PDR_FP64 ? 0.0 : 1.0) +
                      8.0 * (6.0 * m + 4.0 * n + 4.0 * K) + 8.0 * (double)(opt.z_log_capacity > 0 ? opt.z_log_capacity : pdr::kZLogCap) +
                      16.0 * (double)pdr::kHeightBlocksMax;
        size_t free_b = 0, total_b = 0;
        e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) {
            c->err = std::string("hipMemGetInfo: ") + hipGetErrorString(e);
            return init_fail(c, PDR_ERR_DEVICE, out);
        }
        if (need > 0.98 * (double)free_b) {
            char buf[160];
            snprintf(buf, sizeof buf, "instance needs %.3g GB of device memory, %.3g GB free",
                     need / 1e9, (double)free_b / 1e9);
            c->err = buf;
            return init_fail(c, PDR_ERR_OOM, out);
        }
    }

    // ---- host-side graph preparation: CSC of in-arcs, degrees, injections
    std::vector<int32_t> rp32(n + 1), in_ptr(n + 1, 0), in_idx(m), inj_ptr(n + 1, 0),
        inj_k(2 * (size_t)K);
    std::vector<double> inj_val(2 * (size_t)K);
    for (int32_t i = 0; i <= n; ++i) rp32[i] = (int32_t)row_ptr[i];
    for (int32_t q = 0; q < m; ++q) in_ptr[col[q] + 1] += 1;
    for (int32_t i = 0; i < n; ++i) in_ptr[i + 1] += in_ptr[i];
    {
        std::vector<int32_t> fill(in_ptr.begin(), in_ptr.end() - 1);
        for (int32_t q = 0; q < m; ++q) in_idx[fill[col[q]]++] = q;  // ascending arc id per head
    }
    for (int32_t k = 0; k < K; ++k) {
        inj_ptr[s[k] + 1] += 1;
        inj_ptr[t[k] + 1] += 1;
    }
    for (int32_t i = 0; i < n; ++i) inj_ptr[i + 1] += inj_ptr[i];
    {
        std::vector<int32_t> fill(inj_ptr.begin(), inj_ptr.end() - 1);
        for (int32_t k = 0; k < K; ++k) {
            inj_k[fill[s[k]]] = k;
            inj_val[fill[s[k]]++] = d[k];
            inj_k[fill[t[k]]] = k;
            inj_val[fill[t[k]]++] = -d[k];
        }
    }

    std::vector<int32_t> vorder, aorder, cstart;
    locality_order(n, rp32.data(), col, in_ptr, in_idx, tails, c->cluster_size, vorder, aorder,
                   cstart);
    {
        // the kernels index through these arrays: they must be permutations
        std::vector<char> hit_v(n, 0), hit_a(m > 0 ? m : 1, 0);
        bool ok = (int64_t)vorder.size() == n && (int64_t)aorder.size() == m;
        for (int32_t v : vorder) ok = ok && v >= 0 && v < n && !hit_v[v] && (hit_v[v] = 1);
        for (int32_t e : aorder) ok = ok && e >= 0 && e < m && !hit_a[e] && (hit_a[e] = 1);
        if (!ok) {
            c->err = "internal error: the visiting order is not a permutation";
            return init_fail(c, PDR_ERR_STATE, out);
        }
    }

    auto oom_or_dev = [&](hipError_t err, const char *what) {
        if (err == hipErrorOutOfMemory) {
            c->err = std::string("out of device memory: ") + what;
            return init_fail(c, PDR_ERR_OOM, out);
        }
        c->err = std::string(what) + ": " + hipGetErrorString(err);
        return init_fail(c, PDR_ERR_DEVICE, out);
    };
#define PDR_UP(ptr, src, cnt)                                  \
    do {                                                       \
        hipError_t _e = upload(c, &(ptr), (src), (size_t)(cnt)); \
        if (_e != hipSuccess) return oom_or_dev(_e, #ptr);     \
    } while (0)
    PDR_UP(c->d_row_ptr, rp32.data(), n + 1);
    PDR_UP(c->d_tails, tails.data(), m);
    PDR_UP(c->d_heads, col, m);
    PDR_UP(c->d_in_ptr, in_ptr.data(), n + 1);
    PDR_UP(c->d_in_idx, in_idx.data(), m);
    PDR_UP(c->d_deg, deg.data(), n);
    PDR_UP(c->d_inj_ptr, inj_ptr.data(), n + 1);
    PDR_UP(c->d_inj_k, inj_k.data(), 2 * (size_t)K);
    PDR_UP(c->d_inj_val, inj_val.data(), 2 * (size_t)K);
    PDR_UP(c->d_u, u, m);
    PDR_UP(c->d_s, s, K);
    PDR_UP(c->d_t, t, K);
    PDR_UP(c->d_d, d, K);
    PDR_UP(c->d_vorder, vorder.data(), n);
    PDR_UP(c->d_aorder, aorder.data(), m);
    {
        // incidence lists in visiting order (in-arcs, then out-arcs, each in
        // ascending id: the summation order of the excess)
        std::vector<int32_t> vinfo(8 * (size_t)n), vinc(2 * (size_t)m > 0 ? 2 * (size_t)m : 1);
        int32_t p = 0;
        for (int32_t pos = 0; pos < n; ++pos) {
            const int32_t i = vorder[pos];
            int32_t *vi = &vinfo[8 * (size_t)pos];
            vi[0] = i;
            vi[1] = p;
            vi[2] = in_ptr[i + 1] - in_ptr[i];
            for (int32_t q = in_ptr[i]; q < in_ptr[i + 1]; ++q) vinc[p++] = in_idx[q];
            for (int32_t e = rp32[i]; e < rp32[i + 1]; ++e) vinc[p++] = e;
            vi[3] = p;
            // injections: the kernel skips them for vectors outside [kmin, kmax]
            vi[4] = inj_ptr[i];
            vi[5] = inj_ptr[i + 1];
            vi[6] = K;
            vi[7] = -1;
            for (int32_t q = inj_ptr[i]; q < inj_ptr[i + 1]; ++q) {
                vi[6] = std::min(vi[6], inj_k[q]);
                vi[7] = std::max(vi[7], inj_k[q]);
            }
        }
        PDR_UP(c->d_vinfo, vinfo.data(), 8 * (size_t)n);
        PDR_UP(c->d_vinc, vinc.data(), vinc.size());
        if (c->req_height_kernel == 2) {
            std::vector<int32_t> tinfo, tarc;
            std::vector<uint16_t> tslot;
            if (build_tiles(m, vinfo, vinc, cstart, pdr::kTileVerts, pdr::kTileArcs, tinfo, tarc,
                            tslot)) {
                c->ntiles = (int32_t)(tinfo.size() / 4);
                if (tarc.empty()) tarc.push_back(0);
                PDR_UP(c->d_tinfo, tinfo.data(), tinfo.size());
                PDR_UP(c->d_tarc, tarc.data(), tarc.size());
                PDR_UP(c->d_tslot, tslot.data(), tslot.size());
            } else {
                c->err = "height_kernel 2: a vertex has more incident arcs than a tile holds (" +
                         std::to_string(pdr::kTileArcs) + ")";
                return init_fail(c, PDR_ERR_INVALID, out);
            }
        }
    }
#undef PDR_UP
    c->g = DevGraph{n,           m,         K,           c->Kp,        0,           0,         0,
                    c->d_row_ptr, c->d_tails, c->d_heads, c->d_in_ptr, c->d_in_idx,
                    c->d_deg,     c->d_inj_ptr, c->d_inj_k, c->d_inj_val, c->d_u,
                    c->d_s,       c->d_t,     c->d_d,       c->d_vorder, c->d_aorder,
                    c->d_vinfo,   c->d_vinc};
    c->g.tinfo = c->d_tinfo;
    c->g.tarc = c->d_tarc;
    c->g.tslot = c->d_tslot;
    set_height_chunk(c);
    set_cache_policy(c);

    pdr_status st = ensure_buffers(c, c->precision);
    if (st != PDR_OK) return init_fail(c, st, out);
    c->nzpart = pdr::kHeightBlocksMax;  // partials of any height grid
#define PDR_AL(ptr, cnt)                                     \
    do {                                                     \
        hipError_t _e = dalloc(c, &(ptr), (size_t)(cnt));    \
        if (_e != hipSuccess) return oom_or_dev(_e, #ptr);   \
    } while (0)
    PDR_AL(c->Fsum, m);
    PDR_AL(c->beta, m);
    PDR_AL(c->zpart, 3 * c->nzpart);
    PDR_AL(c->maxpart, c->nzpart);
    PDR_AL(c->arcpart, 3 * (size_t)m);
    PDR_AL(c->resout, 8);
    PDR_AL(c->zlog, c->zlog_cap);
    PDR_AL(c->ctrl, 1);
#undef PDR_AL
    e = hipHostMalloc((void **)&c->h_ctrl, sizeof(Ctrl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_res, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return oom_or_dev(e, "hipHostMalloc");

    // ---- initial state: f = 0, v = 0, beta = beta_init, t = 0, z_prev = +inf
    // (Algorithms 1, 3, 4)
    const size_t mK = (size_t)m * c->Kp;
    void *f = cur_f(c);
    e = hipMemsetAsync(f, 0, mK * (c->precision == PDR_FP64 ? 8 : 4), c->stream);
    if (e == hipSuccess && c->method == PDR_GDM)
        e = hipMemsetAsync(cur_v(c), 0, mK * (c->precision == PDR_FP64 ? 8 : 4), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->Fsum, 0, (size_t)(m ? m : 1) * 8, c->stream);
    if (e != hipSuccess) return oom_or_dev(e, "hipMemsetAsync");
    {
        std::vector<double> b(m > 0 ? m : 1, c->agd.beta_init);
        e = hipMemcpyAsync(c->beta, b.data(), b.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return oom_or_dev(e, "beta upload");
        std::memset(c->h_ctrl, 0, sizeof(Ctrl));
        c->h_ctrl->z_prev = std::numeric_limits<double>::infinity();
        e = hipMemcpyAsync(c->ctrl, c->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return oom_or_dev(e, "state upload");
    }
    *out = c;
    return PDR_OK;
}

static pdr_status pdr_sweep_body(pdr_ctx *c, int64_t max_sweeps, double eps_obj, double z_target)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (max_sweeps < 0) return fail(c, PDR_ERR_INVALID, "max_sweeps must be >= 0");
    if (std::isnan(eps_obj) || std::isnan(z_target))
        return fail(c, PDR_ERR_INVALID, "eps_obj and z_target must not be NaN");
    PDR_CHECK(c, pdr::launch_begin(c->ctrl, eps_obj, z_target, c->stream));
    const bool poll = eps_obj > 0.0 || z_target > 0.0;
    const int64_t G = c->graph_sweeps;
    hipGraphExec_t ge = nullptr;
    if (G > 0 && max_sweeps >= G) {
        st = sweep_graph(c, &ge);
        if (st != PDR_OK) return st;
    }
    int64_t batch = 16, since = 0, s = 0;
    while (s < max_sweeps) {
        if (ge && max_sweeps - s >= G) {
            PDR_CHECK(c, hipGraphLaunch(ge, c->stream));
            s += G;
            since += G;
        } else {
            PDR_CHECK(c, enqueue_passes(c, 1, c->stream));
            s += 1;
            since += 1;
        }
        if (poll && since >= batch && s < max_sweeps) {
            since = 0;
            if (batch < 1024) batch *= 2;
            st = sync_ctrl(c);
            if (st != PDR_OK) return st;
            if (c->h_ctrl->stopped) break;
        }
    }
    return PDR_OK;
}

static pdr_status pdr_solve_body(pdr_ctx *c, double z_target, int64_t max_sweeps, int64_t window,
                                 double floor_factor, int64_t *sweeps_fp32, int64_t *sweeps_fp64)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!(z_target > 0.0) || max_sweeps < 0 || window < 1 || std::isnan(floor_factor))
        return fail(c, PDR_ERR_INVALID, "need z_target > 0, max_sweeps >= 0, window >= 1");
    const double kappa = floor_factor > 0.0 ? floor_factor
                         : c->method == PDR_GDM ? kFloorFactorGdm : kFloorFactor;
    int64_t n32 = 0, n64 = 0, total = 0;
    // the hand-over tracking continues where the previous call left it
    double &best_before = c->solve_track.best_before;
    int &stalled = c->solve_track.stalled;  // consecutive windows without a new lowest z
    // lowest z and passes of the recent FP32 windows (the descent rate is
    // measured over kRateWindows of them)
    std::vector<std::pair<double, int64_t>> &recent = c->solve_track.recent;
    std::vector<double> zl;
    while (total < max_sweeps) {
        st = sync_ctrl(c);
        if (st != PDR_OK) return st;
        const int64_t t0 = c->h_ctrl->t, ev0 = c->h_ctrl->evals;
        const int64_t chunk = std::min(window, max_sweeps - total);
        st = pdr_sweep(c, chunk, 0.0, z_target);
        if (st != PDR_OK) return st;
        st = sync_ctrl(c);
        if (st != PDR_OK) return st;
        const int64_t ran = c->h_ctrl->t - t0, nev = c->h_ctrl->evals - ev0;
        (c->precision == PDR_FP64 ? n64 : n32) += ran;
        total += ran;
        if (c->h_ctrl->numeric) return fail(c, PDR_ERR_NUMERIC, "the objective is not finite");
        if (c->h_ctrl->stopped || ran == 0) break;
        if (c->precision == PDR_FP32_BULK && nev > 1) {
            zl.resize((size_t)nev);
            st = pdr_z_log(c, ev0, nev, zl.data());
            if (st != PDR_OK) return st;
            const double cur = *std::min_element(zl.begin(), zl.end());
            // FP32 rounding adds noise of size z_noise every pass; a descent that
            // shrinks z by the factor (1 - rate) per pass settles where the two
            // balance, near z_noise / rate. Hand over at kappa times that
            // level, or when the objective stalls. The rate is that of the
            // windows' lowest z over the last kRateWindows windows: GDM's z is
            // not monotone, so the ends of one window say little.
            recent.emplace_back(cur, ran);
            if ((int)recent.size() > kRateWindows + 1) recent.erase(recent.begin());
            double rate = 0.0;
            if ((int)recent.size() == kRateWindows + 1 && cur > 0.0 && cur < recent.front().first) {
                int64_t span = 0;
                for (size_t q = 1; q < recent.size(); ++q) span += recent[q].second;
                rate = std::log(recent.front().first / cur) / (double)std::max<int64_t>(span, 1);
            }
            const bool near_floor = rate > 0.0 && cur <= kappa * (c->h_ctrl->z_noise / rate);
            // a stall is kStallWindows windows in a row without a new lowest z
            // by more than the FP32 noise could account for (GDM's objective is
            // not monotone: one window can miss the last trough and still be on
            // the way down; a slow but steady descent, as AGD's at 10^4
            // commodities, gains far more than the noise per window)
            // (the first window after a start or a reset has nothing to beat)
            const bool progress =
                !std::isfinite(best_before) ||
                cur < best_before - std::max(kStallNoise * c->h_ctrl->z_noise, 1e-12 * best_before);
            stalled = progress ? 0 : stalled + 1;
            const double best_now = std::min(best_before, cur);
            if (near_floor || stalled >= kStallWindows) {
                st = pdr_set_precision(c, PDR_FP64);  // also resets the tracking
                if (st != PDR_OK) return st;
            } else {
                best_before = best_now;
            }
        }
    }
    if (sweeps_fp32) *sweeps_fp32 = n32;
    if (sweeps_fp64) *sweeps_fp64 = n64;
    return PDR_OK;
}

static pdr_status pdr_profile_sweeps_body(pdr_ctx *c, int64_t sweeps, double *kernel_ms)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (sweeps < 0 || !kernel_ms) return fail(c, PDR_ERR_INVALID, "bad arguments");
    const bool fp64 = c->precision == PDR_FP64;
    void *f = cur_f(c);
    void *h = cur_h(c);
    const pdr::AgdParams prm = agd_params(c);
    constexpr int B = 64;  // sweeps per batch of events
    hipEvent_t ev[B][3];
    for (int q = 0; q < B; ++q)
        for (int r = 0; r < 3; ++r) PDR_CHECK(c, hipEventCreate(&ev[q][r]));
    double tot[2] = {0.0, 0.0};
    hipError_t err = pdr::launch_begin(c->ctrl, 0.0, 0.0, c->stream);
    for (int64_t s0 = 0; s0 < sweeps && err == hipSuccess; s0 += B) {
        const int nb = (int)std::min<int64_t>(B, sweeps - s0);
        for (int q = 0; q < nb && err == hipSuccess; ++q) {
            err = hipEventRecord(ev[q][0], c->stream);
            if (err == hipSuccess)
                err = pdr::launch_height(c->g, fp64, f, h, c->zpart, c->Fsum, c->ctrl, c->zlog,
                                         c->zlog_cap - 1,
                                         c->stream);
            if (err == hipSuccess) err = hipEventRecord(ev[q][1], c->stream);
            if (err == hipSuccess)
                err = c->method == PDR_ESO || c->method == PDR_CAP
                          ? pdr::launch_eso(c->g, fp64, c->tiling, f, h, c->Fsum, c->ctrl,
                                            c->method == PDR_CAP, c->stream)
                          : pdr::launch_agd(c->g, fp64, c->tiling, f, h, c->Fsum, c->beta, prm,
                                            c->ctrl, c->method == PDR_GDM ? cur_v(c) : nullptr,
                                            c->stream);
            if (err == hipSuccess) err = hipEventRecord(ev[q][2], c->stream);
        }
        if (err == hipSuccess) err = hipEventSynchronize(ev[nb - 1][2]);
        for (int q = 0; q < nb && err == hipSuccess; ++q)
            for (int r = 0; r < 2 && err == hipSuccess; ++r) {
                float ms = 0.0f;
                err = hipEventElapsedTime(&ms, ev[q][r], ev[q][r + 1]);
                tot[r] += ms;
            }
    }
    for (int q = 0; q < B; ++q)
        for (int r = 0; r < 3; ++r) (void)hipEventDestroy(ev[q][r]);
    PDR_CHECK(c, err);
    kernel_ms[0] = tot[0];
    kernel_ms[1] = tot[1];
    return PDR_OK;
}

static pdr_status pdr_residual_body(pdr_ctx *c, pdr_residual_t *out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!out) return fail(c, PDR_ERR_INVALID, "out is NULL");
    const bool fp64 = c->precision == PDR_FP64;
    void *f = cur_f(c);
    PDR_CHECK(c, pdr::launch_height_resid(c->g, fp64, f, c->h64, c->zpart, c->maxpart, c->stream));
    PDR_CHECK(c, pdr::launch_resid(c->g, fp64, f, c->h64, c->Fsum, c->zpart,
                                   pdr::height_blocks(c->g, fp64 ? 8 : 4), c->maxpart, c->arcpart,
                                   c->resout, c->stream));
    PDR_CHECK(c, hipMemcpyAsync(c->h_res, c->resout, 8 * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
    st = sync_ctrl(c);
    if (st != PDR_OK) return st;
    const double *r = c->h_res;
    out->z = r[0];
    out->z_psi = r[1];
    out->z_h = r[2];
    out->kkt_sq = r[3];
    out->max_abs_excess = r[4];
    out->max_congestion = r[5];
    out->farkas_gap = r[6];
    out->farkas_tol = r[7];
    out->z_fp32_floor = c->precision == PDR_FP32_BULK ? c->h_ctrl->z_noise : 0.0;
    out->sweeps_done = c->h_ctrl->t;
    out->evaluations = c->h_ctrl->evals;
    out->stopped = c->h_ctrl->stopped;
    if (r[6] > r[7])
        out->verdict = PDR_INFEASIBLE;
    else if (r[0] <= c->z_feasible_tol)
        out->verdict = PDR_FEASIBLE;
    else
        out->verdict = PDR_UNDECIDED;
    if (!std::isfinite(r[0]) || c->h_ctrl->numeric)
        return fail(c, PDR_ERR_NUMERIC, "the objective is not finite");
    return PDR_OK;
}

static pdr_status pdr_flows_body(pdr_ctx *c, double *host_out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!host_out) return fail(c, PDR_ERR_INVALID, "host_out is NULL");
    if (c->m == 0) return PDR_OK;
    const size_t K = c->K, Kp = c->Kp, m = c->m;
    if (c->precision == PDR_FP64) {
        PDR_CHECK(c, hipMemcpy2DAsync(host_out, K * 8, c->f64, Kp * 8, K * 8, m,
                                      hipMemcpyDeviceToHost, c->stream));
        PDR_CHECK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(m * K);
        PDR_CHECK(c, hipMemcpy2DAsync(tmp.data(), K * 4, c->f32, Kp * 4, K * 4, m,
                                      hipMemcpyDeviceToHost, c->stream));
        PDR_CHECK(c, hipStreamSynchronize(c->stream));
        for (size_t q = 0; q < m * K; ++q) host_out[q] = (double)tmp[q];
    }
    return PDR_OK;
}

static pdr_status pdr_flows_device_body(pdr_ctx *c, void *dev_out, int32_t fp64)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!dev_out) return fail(c, PDR_ERR_INVALID, "dev_out is NULL");
    if (c->m == 0) return PDR_OK;
    PDR_CHECK(c, pdr::launch_unpad(c->g, cur_f(c), c->precision == PDR_FP64, dev_out, fp64 != 0,
                                   c->stream));
    return PDR_OK;
}

static pdr_status pdr_heights_body(pdr_ctx *c, double *host_out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!host_out) return fail(c, PDR_ERR_INVALID, "host_out is NULL");
    const bool fp64 = c->precision == PDR_FP64;
    PDR_CHECK(c, pdr::launch_height_resid(c->g, fp64, cur_f(c), c->h64, c->zpart, c->maxpart,
                                          c->stream));
    const size_t K = c->K, Kp = c->Kp;
    PDR_CHECK(c, hipMemcpy2DAsync(host_out, K * 8, c->h64, Kp * 8, K * 8, (size_t)c->n,
                                  hipMemcpyDeviceToHost, c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}

static pdr_status pdr_learning_rates_body(pdr_ctx *c, double *host_out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (!host_out) return fail(c, PDR_ERR_INVALID, "host_out is NULL");
    if (c->m == 0) return PDR_OK;
    PDR_CHECK(c, hipMemcpyAsync(host_out, c->beta, (size_t)c->m * 8, hipMemcpyDeviceToHost,
                                c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}

static pdr_status pdr_velocities_body(pdr_ctx *c, double *host_out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (c->method != PDR_GDM) return fail(c, PDR_ERR_STATE, "velocities exist for PDR_GDM only");
    if (!host_out) return fail(c, PDR_ERR_INVALID, "host_out is NULL");
    if (c->m == 0) return PDR_OK;
    const size_t K = c->K, Kp = c->Kp, m = c->m;
    if (c->precision == PDR_FP64) {
        PDR_CHECK(c, hipMemcpy2DAsync(host_out, K * 8, c->v64, Kp * 8, K * 8, m,
                                      hipMemcpyDeviceToHost, c->stream));
        PDR_CHECK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(m * K);
        PDR_CHECK(c, hipMemcpy2DAsync(tmp.data(), K * 4, c->v32, Kp * 4, K * 4, m,
                                      hipMemcpyDeviceToHost, c->stream));
        PDR_CHECK(c, hipStreamSynchronize(c->stream));
        for (size_t q = 0; q < m * K; ++q) host_out[q] = (double)tmp[q];
    }
    return PDR_OK;
}

static pdr_status pdr_z_log_body(pdr_ctx *c, int64_t first, int64_t count, double *host_out)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (count < 0 || first < 0 || (count > 0 && !host_out))
        return fail(c, PDR_ERR_INVALID, "bad z log range");
    st = sync_ctrl(c);
    if (st != PDR_OK) return st;
    const int64_t evals = c->h_ctrl->evals;
    if (first + count > evals || first < evals - c->zlog_cap)
        return fail(c, PDR_ERR_INVALID, "z log range not available");
    int64_t done = 0;
    while (done < count) {
        const int64_t pos = (first + done) & (c->zlog_cap - 1);
        int64_t len = std::min<int64_t>(count - done, c->zlog_cap - pos);
        PDR_CHECK(c, hipMemcpyAsync(host_out + done, c->zlog + pos, (size_t)len * 8,
                                    hipMemcpyDeviceToHost, c->stream));
        done += len;
    }
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}

static pdr_status pdr_set_precision_body(pdr_ctx *c, int32_t precision)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (c->batch_member)
        return fail(c, PDR_ERR_STATE, "a batch member switches precision with its batch");
    return set_precision_impl(c, precision);
}

}  // extern "C"

namespace pdr_host {
void set_cache_policy(pdr_ctx *c)
{
    const double w = c->precision == PDR_FP64 ? 8.0 : 4.0;
    double bytes = w * ((double)c->m + (double)c->n) * (double)c->Kp;
    if (c->method == PDR_GDM) bytes += w * (double)c->m * (double)c->Kp;
    bool temporal = bytes <= kCacheResidentBytes;
    if (c->req_cache_policy == 1) temporal = true;
    if (c->req_cache_policy == 2) temporal = false;
    c->g.temporal = (temporal && !c->batch_member) ? 1 : 0;
    // the tiled height kernel only on request: it reads less but runs slower
    c->g.ntiles = c->req_height_kernel == 2 ? c->ntiles : 0;
}

pdr_status check_state_args(pdr_ctx *c, const double *f, const double *beta, const double *v,
                            int64_t t, double z_prev)
{
    if (!f && c->m > 0) return fail(c, PDR_ERR_INVALID, "f is NULL");
    if (t < 0) return fail(c, PDR_ERR_INVALID, "t must be >= 0");
    if (std::isnan(z_prev)) return fail(c, PDR_ERR_INVALID, "z_prev is NaN");
    const size_t mK = (size_t)c->m * c->K;
    for (size_t q = 0; q < mK; ++q)
        if (!finite_nonneg(f[q])) return fail(c, PDR_ERR_INVALID, "flows must be finite and >= 0");
    if (beta)
        for (int32_t e = 0; e < c->m; ++e)
            if (!(beta[e] > 0) || !std::isfinite(beta[e]))
                return fail(c, PDR_ERR_INVALID, "learning rates must be finite and > 0");
    if (v && c->method == PDR_GDM)
        for (size_t q = 0; q < mK; ++q)
            if (!std::isfinite(v[q])) return fail(c, PDR_ERR_INVALID, "velocities must be finite");
    return PDR_OK;
}

// Upload host rows (m x K, unpadded) into a padded device array through a
// staging buffer of `cap` doubles, in chunks of whole rows.
static pdr_status stage_rows(pdr_ctx *c, const double *src, void *dst, double *staging,
                             int64_t cap)
{
    const int64_t K = c->K, m = c->m;
    const int64_t per = cap / K;  // rows per chunk (>= 1: checked by the caller)
    for (int64_t r0 = 0; r0 < m; r0 += per) {
        const int64_t rows = std::min(per, m - r0);
        PDR_CHECK(c, hipMemcpyAsync(staging, src + r0 * K, (size_t)(rows * K) * 8,
                                    hipMemcpyHostToDevice, c->stream));
        PDR_CHECK(c, pdr::launch_pad_rows(c->g, staging, dst, c->precision == PDR_FP64, r0, rows,
                                          c->stream));
    }
    return PDR_OK;
}

pdr_status set_state_impl(pdr_ctx *c, const double *f, const double *beta, const double *v,
                          int64_t t, double z_prev, double *staging, int64_t staging_doubles)
{
    c->solve_track = pdr_ctx::SolveTrack{};
    if (c->m > 0) {
        if (staging_doubles < c->K)
            return fail(c, PDR_ERR_INVALID, "one arc row does not fit the staging buffer");
        pdr_status st = stage_rows(c, f, cur_f(c), staging, staging_doubles);
        if (st != PDR_OK) return st;
        PDR_CHECK(c, pdr::launch_rowsum(c->g, c->precision == PDR_FP64, c->tiling, cur_f(c),
                                        c->Fsum, c->stream));
        if (v && c->method == PDR_GDM) {
            st = stage_rows(c, v, cur_v(c), staging, staging_doubles);
            if (st != PDR_OK) return st;
        }
        if (beta)
            PDR_CHECK(c, hipMemcpyAsync(c->beta, beta, (size_t)c->m * 8, hipMemcpyHostToDevice,
                                        c->stream));
        PDR_CHECK(c, hipStreamSynchronize(c->stream));
    }
    pdr_status st = sync_ctrl(c);
    if (st != PDR_OK) return st;
    c->h_ctrl->t = t;
    c->h_ctrl->z_prev = z_prev;
    c->h_ctrl->stopped = 0;
    c->h_ctrl->numeric = 0;
    return push_ctrl(c);
}

pdr_status set_precision_impl(pdr_ctx *c, int32_t precision)
{
    pdr_status st;
    if (precision != PDR_FP64 && precision != PDR_FP32_BULK)
        return fail(c, PDR_ERR_INVALID, "unknown precision");
    if (precision == c->precision) return PDR_OK;
    Tiling tl;
    st = choose_tiling(c, precision, &tl);
    if (st != PDR_OK) return st;
    st = ensure_buffers(c, precision);
    if (st != PDR_OK) return st;
    const int64_t mK = (int64_t)c->m * c->Kp;
    if (precision == PDR_FP64)
        PDR_CHECK(c, pdr::launch_convert(c->f32, false, c->f64, true, mK, c->stream));
    else
        PDR_CHECK(c, pdr::launch_convert(c->f64, true, c->f32, false, mK, c->stream));
    if (c->method == PDR_GDM) {
        if (precision == PDR_FP64)
            PDR_CHECK(c, pdr::launch_convert(c->v32, false, c->v64, true, mK, c->stream));
        else
            PDR_CHECK(c, pdr::launch_convert(c->v64, true, c->v32, false, mK, c->stream));
    }
    c->precision = precision;
    c->tiling = tl;
    c->solve_track = pdr_ctx::SolveTrack{};
    set_height_chunk(c);
    set_cache_policy(c);
    PDR_CHECK(c, pdr::launch_rowsum(c->g, precision == PDR_FP64, c->tiling, cur_f(c), c->Fsum,
                                    c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    return PDR_OK;
}
}  // namespace pdr_host

extern "C" {

static pdr_status pdr_set_state_body(pdr_ctx *c, const double *f, const double *beta,
                                     const double *v, int64_t t, double z_prev)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    st = check_state_args(c, f, beta, v, t, z_prev);
    if (st != PDR_OK) return st;
    const size_t mK = (size_t)c->m * c->K;
    double *staging = nullptr;
    if (mK > 0) {  // one staging buffer for the whole state
        hipError_t e = hipMalloc((void **)&staging, mK * 8);
        if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (staging)");
        PDR_CHECK(c, e);
    }
    st = set_state_impl(c, f, beta, v, t, z_prev, staging, (int64_t)mK);
    if (staging) (void)hipFree(staging);
    return st;
}

static pdr_status pdr_stream_body(const pdr_ctx *c, void **stream)
{
    if (!c || !stream) return PDR_ERR_INVALID;
    *stream = (void *)c->stream;
    return PDR_OK;
}

pdr_status pdr_tiling(const pdr_ctx *c, int32_t *lanes_per_arc, int32_t *vec_per_lane, int32_t *Kp)
{
    if (!c) return PDR_ERR_INVALID;
    if (lanes_per_arc) *lanes_per_arc = c->tiling.lanes;
    if (vec_per_lane) *vec_per_lane = c->tiling.nv;
    if (Kp) *Kp = c->Kp;
    return PDR_OK;
}

static pdr_status pdr_adjoint_body(pdr_ctx *c, int64_t T, int32_t checkpoint, double *z_out,
                                   double *grad_u, double *grad_d)
{
    pdr_status st;
    if (!usable(c, &st)) return st;
    if (T < 0 || checkpoint < 0 || !z_out || (c->m > 0 && !grad_u) || !grad_d)
        return fail(c, PDR_ERR_INVALID, "need T >= 0, checkpoint >= 0 and output arrays");
    if (c->method != PDR_ESO || c->precision != PDR_FP64)
        return fail(c, PDR_ERR_STATE, "the adjoint needs a PDR_ESO context in PDR_FP64");
    if (c->tiling.nv < 0)
        return fail(c, PDR_ERR_STATE,
                    "the adjoint holds arc rows in registers: at most 16,384 commodities");
    const int64_t C = checkpoint > 0 ? checkpoint : 16;
    const int64_t nseg = (T + C - 1) / C;
    const size_t mK = (size_t)c->m * c->Kp, nK = (size_t)c->n * c->Kp;
    // working memory, released on every return
    struct Bufs {
        std::vector<void *> p;
        ~Bufs()
        {
            for (void *q : p) (void)hipFree(q);
        }
        hipError_t get(double **out, size_t count)
        {
            p.push_back(nullptr);  // the slot first, so a failed push leaks nothing
            hipError_t e = hipMalloc(&p.back(), (count ? count : 1) * sizeof(double));
            *out = e == hipSuccess ? (double *)p.back() : nullptr;
            return e;
        }
    } bufs;
    // ckpt[j] = f^(jC); seg / hseg: a segment's recomputed flows f^(a+1 .. b-1)
    // and heights h^(a .. b-1)
    const size_t segC = (size_t)std::min<int64_t>(C, std::max<int64_t>(T, 1));
    std::vector<double *> ckpt((size_t)nseg), seg(segC > 1 ? segC - 1 : 0), hseg(T > 0 ? segC : 0);
    double *cbar = nullptr, *Dbar = nullptr, *ubar = nullptr, *dbar = nullptr;
    hipError_t e = hipSuccess;
    for (auto &x : ckpt)
        if (e == hipSuccess) e = bufs.get(&x, mK);
    for (auto &x : seg)
        if (e == hipSuccess) e = bufs.get(&x, mK);
    for (auto &x : hseg)
        if (e == hipSuccess) e = bufs.get(&x, nK);
    if (e == hipSuccess) e = bufs.get(&cbar, mK);
    if (e == hipSuccess) e = bufs.get(&Dbar, nK);
    if (e == hipSuccess) e = bufs.get(&ubar, (size_t)c->m);
    if (e == hipSuccess) e = bufs.get(&dbar, (size_t)c->K);
    if (e == hipErrorOutOfMemory) return fail(c, PDR_ERR_OOM, "out of device memory (adjoint)");
    PDR_CHECK(c, e);
    double *f = c->f64;
    // ---- forward: T passes as pdr_sweep runs them, f kept every C passes
    PDR_CHECK(c, pdr::launch_begin(c->ctrl, 0.0, 0.0, c->stream));
    for (int64_t t = 0; t < T; ++t) {
        if (t % C == 0)
            PDR_CHECK(c, hipMemcpyAsync(ckpt[(size_t)(t / C)], f, mK * 8, hipMemcpyDeviceToDevice,
                                        c->stream));
        PDR_CHECK(c, enqueue_passes(c, 1, c->stream));
    }
    // ---- z(f^T) and the seed dz/df, dz/du, dz/dd at f^T (pdr_residual leaves
    // the FP64 heights of f^T in h64)
    pdr_residual_t res;
    st = pdr_residual(c, &res);
    if (st != PDR_OK) return st;  // PDR_ERR_NUMERIC: z(f^T) is not finite
    PDR_CHECK(c, pdr::launch_adj_seed(c->g, c->Fsum, c->h64, cbar, ubar, dbar, c->stream));
    PDR_CHECK(c, hipMemsetAsync(Dbar, 0, nK * 8, c->stream));
    // ---- reverse, segment by segment from the last: recompute the segment's
    // flows and heights once, then reverse its passes
    for (int64_t j = nseg - 1; j >= 0; --j) {
        const int64_t a = j * C, b = std::min(T, a + C);
        const double *prev = ckpt[(size_t)j];
        for (int64_t k = 0; k < b - a; ++k) {  // h^(a+k), then f^(a+k+1) if inside
            PDR_CHECK(c, pdr::launch_height_resid(c->g, true, prev, hseg[(size_t)k], c->zpart,
                                                  c->maxpart, c->stream));
            if (k + 1 < b - a) {
                double *nxt = seg[(size_t)k];
                PDR_CHECK(c, pdr::launch_eso_oop(c->g, c->tiling, prev, nxt, hseg[(size_t)k],
                                                 c->Fsum, c->stream));
                prev = nxt;
            }
        }
        for (int64_t t = b - 1; t >= a; --t) {
            const double *ft = t == a ? ckpt[(size_t)j] : seg[(size_t)(t - a - 1)];
            PDR_CHECK(c, pdr::launch_adj_pass(c->g, c->tiling, ft, hseg[(size_t)(t - a)], cbar,
                                              Dbar, ubar, dbar, c->stream));
        }
    }
    // the recomputation overwrote the row sums and heights: restore them for f^T
    PDR_CHECK(c, pdr::launch_rowsum(c->g, true, c->tiling, f, c->Fsum, c->stream));
    PDR_CHECK(c, pdr::launch_height_resid(c->g, true, f, c->h64, c->zpart, c->maxpart, c->stream));
    if (c->m > 0)
        PDR_CHECK(c, hipMemcpyAsync(grad_u, ubar, (size_t)c->m * 8, hipMemcpyDeviceToHost,
                                    c->stream));
    PDR_CHECK(c, hipMemcpyAsync(grad_d, dbar, (size_t)c->K * 8, hipMemcpyDeviceToHost, c->stream));
    PDR_CHECK(c, hipStreamSynchronize(c->stream));
    *z_out = res.z;
    return PDR_OK;
}

static pdr_status pdr_measure_copy_body(int64_t bytes, int32_t iters, double *gbps)
{
    if (bytes < 16 || iters < 1 || !gbps) {
        g_init_error = "pdr_measure_copy: need bytes >= 16, iters >= 1, gbps";
        return PDR_ERR_INVALID;
    }
    const int64_t n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, (size_t)n16 * 16);
    if (e == hipSuccess) e = hipMalloc(&b, (size_t)n16 * 16);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, (size_t)n16 * 16, st);
    if (e == hipSuccess) e = pdr::launch_copy(a, b, n16, st);  // warm up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int q = 0; q < iters && e == hipSuccess; ++q)
        e = pdr::launch_copy(q % 2 ? b : a, q % 2 ? a : b, n16, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) *gbps = 2.0 * (double)n16 * 16.0 * iters / (ms * 1e-3) / 1e9;
    const hipError_t err = e;
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (b) (void)hipFree(b);
    if (a) (void)hipFree(a);
    if (err == hipErrorOutOfMemory) {
        g_init_error = "pdr_measure_copy: out of device memory";
        return PDR_ERR_OOM;
    }
    if (err != hipSuccess) {
        g_init_error = std::string("pdr_measure_copy: ") + hipGetErrorString(err);
        return PDR_ERR_DEVICE;
    }
    return PDR_OK;
}

static void pdr_destroy_body(pdr_ctx *c)
{
    if (!c || c->batch_member) return;  // a batch frees its own members
    (void)hipSetDevice(c->device);
    free_all(c);
    delete c;
}

}  // extern "C"

// ------------------------------------------------------------------ exported entry points
// Each runs its body behind the exception barrier (abi_guard).
extern "C" {

pdr_status pdr_init(pdr_ctx **out, int32_t n, int32_t m, const int64_t *row_ptr,
                    const int32_t *col, const double *u, int32_t K, const int32_t *s,
                    const int32_t *t, const double *d, const pdr_options *opt_in)
{
    pdr_ctx *created = nullptr;
    bool returned = false;
    const pdr_status st = abi_guard(nullptr, nullptr, [&] {
        const pdr_status r = pdr_init_body(out, n, m, row_ptr, col, u, K, s, t, d, opt_in,
                                           &created);
        returned = true;
        return r;
    });
    if (!returned) {  // left part way by an exception: free what was built
        if (created) {
            free_all(created);
            delete created;
        }
        if (out) *out = nullptr;
    }
    return st;
}

pdr_status pdr_sweep(pdr_ctx *c, int64_t max_sweeps, double eps_obj, double z_target)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_sweep_body(c, max_sweeps, eps_obj, z_target); });
}

pdr_status pdr_solve(pdr_ctx *c, double z_target, int64_t max_sweeps, int64_t window,
                     double floor_factor, int64_t *sweeps_fp32, int64_t *sweeps_fp64)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_solve_body(c, z_target, max_sweeps, window, floor_factor, sweeps_fp32, sweeps_fp64); });
}

pdr_status pdr_profile_sweeps(pdr_ctx *c, int64_t sweeps, double *kernel_ms)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_profile_sweeps_body(c, sweeps, kernel_ms); });
}

pdr_status pdr_residual(pdr_ctx *c, pdr_residual_t *out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_residual_body(c, out); });
}

pdr_status pdr_flows(pdr_ctx *c, double *host_out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_flows_body(c, host_out); });
}

pdr_status pdr_flows_device(pdr_ctx *c, void *dev_out, int32_t fp64)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_flows_device_body(c, dev_out, fp64); });
}

pdr_status pdr_stream(const pdr_ctx *c, void **stream)
{
    return abi_guard(nullptr, nullptr, [&] { return pdr_stream_body(c, stream); });
}

pdr_status pdr_heights(pdr_ctx *c, double *host_out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_heights_body(c, host_out); });
}

pdr_status pdr_learning_rates(pdr_ctx *c, double *host_out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_learning_rates_body(c, host_out); });
}

pdr_status pdr_velocities(pdr_ctx *c, double *host_out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_velocities_body(c, host_out); });
}

pdr_status pdr_z_log(pdr_ctx *c, int64_t first, int64_t count, double *host_out)
{
    return abi_guard(c ? &c->err : nullptr, nullptr,
                     [&] { return pdr_z_log_body(c, first, count, host_out); });
}

pdr_status pdr_set_precision(pdr_ctx *c, int32_t precision)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_set_precision_body(c, precision); });
}

pdr_status pdr_set_state(pdr_ctx *c, const double *f, const double *beta, const double *v,
                         int64_t t, double z_prev)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_set_state_body(c, f, beta, v, t, z_prev); });
}

pdr_status pdr_adjoint(pdr_ctx *c, int64_t T, int32_t checkpoint, double *z_out, double *grad_u,
                       double *grad_d)
{
    return abi_guard(c ? &c->err : nullptr, c ? &c->poisoned : nullptr,
                     [&] { return pdr_adjoint_body(c, T, checkpoint, z_out, grad_u, grad_d); });
}

pdr_status pdr_measure_copy(int64_t bytes, int32_t iters, double *gbps)
{
    return abi_guard(nullptr, nullptr, [&] { return pdr_measure_copy_body(bytes, iters, gbps); });
}

void pdr_destroy(pdr_ctx *c)
{
    try {
        pdr_destroy_body(c);
    } catch (...) {  // teardown cannot report; nothing may leave the ABI
    }
}

}  // extern "C"
