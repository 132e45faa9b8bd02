// Kernels and launchers of the sweep's control, height, objective, residual,
// copy and adjoint-vertex steps (non-arc work), and the batched height pass.
#include "pdr_device.h"

namespace pdr {

// ----------------------------------------------------------------- control
__global__ void k_begin(Ctrl *ctrl, double eps_obj, double z_target)
{
    if (threadIdx.x == 0) {
        ctrl->stopped = 0;
        ctrl->eps_obj = eps_obj;
        ctrl->z_target = z_target;
    }
}

__global__ void kb_begin(const InstView *__restrict__ views, int B, double eps_obj,
                         double z_target)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) {
        Ctrl *c = views[b].ctrl;
        c->stopped = 0;
        c->eps_obj = eps_obj;
        c->z_target = z_target;
    }
}


__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ zpart, int nz,
                                                 Ctrl *__restrict__ ctrl,
                                                 double *__restrict__ zlog, int64_t zmask)
{
    reduce_core(zpart, nz, ctrl, zlog, zmask);
}

// Batched: block b reduces instance b's partials into its own control record.
__global__ __launch_bounds__(1024) void kb_reduce(const InstView *__restrict__ views)
{
    const InstView &I = views[blockIdx.x];
    reduce_core(I.zpart, I.nzpart, I.ctrl, I.zlog, I.zmask);
}

// out: z, z_psi, z_h, kkt_sq, max|Delta|, max psi, Farkas gap G, margin tau.
__global__ __launch_bounds__(1024) void k_resid_final(DevGraph g, const double *__restrict__ h64,
                                                      const double *__restrict__ zpart,
                                                      int64_t nz,
                                                      const double *__restrict__ maxpart,
                                                      const double *__restrict__ arcpart,
                                                      double *__restrict__ out)
{
    __shared__ double sh[8][16];
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // zh, zpsi, kkt, ul, maxD, maxpsi, dh, dh_abs
    for (int64_t q = threadIdx.x; q < nz; q += 1024) {
        a[0] += zpart[q];
        a[4] = fmax(a[4], maxpart[q]);
    }
    for (int q = threadIdx.x; q < g.m; q += 1024) {
        const double p = arcpart[2 * (int64_t)g.m + q];
        a[1] += p * p;
        a[2] += arcpart[q];
        a[3] += arcpart[g.m + q];
        a[5] = fmax(a[5], p);
    }
    const int64_t Kp = g.Kp;
    for (int k = threadIdx.x; k < g.K; k += 1024) {
        const double gg = h64[(int64_t)g.s[k] * Kp + k] - h64[(int64_t)g.t[k] * Kp + k];
        a[6] += g.d[k] * gg;
        a[7] += g.d[k] * fabs(gg);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = (q == 4 || q == 5) ? wave_max(a[q]) : wave_sum(a[q]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 8; ++q) sh[q][w] = a[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[8];
        for (int q = 0; q < 8; ++q) {
            double s = sh[q][0];
            for (int ww = 1; ww < 16; ++ww) s = (q == 4 || q == 5) ? fmax(s, sh[q][ww]) : s + sh[q][ww];
            r[q] = s;
        }
        const double zh = 0.5 * r[0], zp = 0.5 * r[1];
        out[0] = zp + zh;
        out[1] = zp;
        out[2] = zh;
        out[3] = r[2];
        out[4] = r[4];
        out[5] = r[5];
        out[6] = r[6] - r[3];
        out[7] = 64.0 * 2.220446049250313e-16 * (r[7] + r[3]);
    }
}

// Plain 16-byte copy, the reference for what HBM delivers to a streaming
// kernel: each block copies contiguous tiles of 4 x 256 vectors with
// non-temporal loads and stores (the fastest of the simple copy shapes on
// this GPU).
__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src,
                                              double2 *__restrict__ dst, int64_t count)
{
    constexpr int U = 4;
    const int64_t tile = 256 * U;
    const int64_t ntiles = count / tile;
    const pdr_d2 *s = reinterpret_cast<const pdr_d2 *>(src);
    pdr_d2 *d = reinterpret_cast<pdr_d2 *>(dst);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * tile + threadIdx.x;
        pdr_d2 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = __builtin_nontemporal_load(s + base + u * 256);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(x[u], d + base + u * 256);
    }
    for (int64_t q = ntiles * tile + (int64_t)blockIdx.x * 256 + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * 256)
        dst[q] = src[q];
}

int64_t height_blocks(const DevGraph &g, int elem_bytes)
{
    const int V = 16 / elem_bytes;
    const int64_t work = (int64_t)g.n * (g.Kp / V);
    int64_t b = work > 0 ? (work + 255) / 256 : 1;
    const int64_t cap = g.height_grid > 0 ? g.height_grid : kHeightBlocksMax;
    return b < cap ? b : cap;
}

hipError_t launch_begin(Ctrl *ctrl, double eps_obj, double z_target, hipStream_t st)
{
    k_begin<<<1, 64, 0, st>>>(ctrl, eps_obj, z_target);
    return hipGetLastError();
}

template <typename T, int U>
static void height_launch(const DevGraph &g, const T *f, T *h, double *zpart, const double *Fsum,
                          Ctrl *ctrl, unsigned nb, hipStream_t st)
{
    if (g.temporal)
        k_height<T, false, U, false><<<nb, 256, 0, st>>>(g, f, h, nullptr, zpart, nullptr, Fsum,
                                                         ctrl);
    else
        k_height<T, false, U, true><<<nb, 256, 0, st>>>(g, f, h, nullptr, zpart, nullptr, Fsum,
                                                        ctrl);
}

// Chunks per unit of the tiled height kernel: about four units per block, so
// the per-unit set-up is spread over many chunks and the last units even out.
static int tile_run(const DevGraph &g, int V, unsigned nb)
{
    const int64_t nchunk = ((int64_t)(g.Kp / V) + kTileVecs - 1) / kTileVecs;
    const int64_t per = 4 * (int64_t)nb;
    int64_t R = ((int64_t)g.ntiles * nchunk + per - 1) / per;
    if (R < 1) R = 1;
    return (int)(R < nchunk ? R : nchunk);
}

template <typename T>
static void height_tiled_launch(const DevGraph &g, const T *f, T *h, double *zpart,
                                const double *Fsum, Ctrl *ctrl, unsigned nb, hipStream_t st)
{
    const int R = tile_run(g, VecT<T>::N, nb);
    if (g.temporal)
        k_height_tiled<T, false><<<nb, kTileThreads, 0, st>>>(g, R, f, h, zpart, Fsum, ctrl);
    else
        k_height_tiled<T, true><<<nb, kTileThreads, 0, st>>>(g, R, f, h, zpart, Fsum, ctrl);
}

hipError_t launch_height(const DevGraph &g, bool fp64, const void *f, void *h, double *zpart,
                         const double *Fsum, Ctrl *ctrl, double *zlog, int64_t zmask,
                         hipStream_t st)
{
    if (g.ntiles > 0) {
        const unsigned nb = (unsigned)g.tile_grid;
        if (fp64)
            height_tiled_launch<double>(g, (const double *)f, (double *)h, zpart, Fsum, ctrl, nb,
                                        st);
        else
            height_tiled_launch<float>(g, (const float *)f, (float *)h, zpart, Fsum, ctrl, nb, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_reduce<<<1, 1024, 0, st>>>(zpart, (int)nb, ctrl, zlog, zmask);
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)height_blocks(g, fp64 ? 8 : 4);
    bool launched = false;
#define PDR_H(U_)                                                                               \
    if (!launched && g.height_unroll == U_) {                                                   \
        if (fp64)                                                                               \
            height_launch<double, U_>(g, (const double *)f, (double *)h, zpart, Fsum, ctrl, nb,  \
                                      st);                                                      \
        else                                                                                    \
            height_launch<float, U_>(g, (const float *)f, (float *)h, zpart, Fsum, ctrl, nb, st); \
        launched = true;                                                                        \
    }
    PDR_HEIGHT_UNROLL(PDR_H)
#undef PDR_H
    if (!launched) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce<<<1, 1024, 0, st>>>(zpart, (int)nb, ctrl, zlog, zmask);
    return hipGetLastError();
}

hipError_t launch_height_resid(const DevGraph &g, bool fp64, const void *f, double *h64,
                               double *zpart, double *maxpart, hipStream_t st)
{
    const unsigned nb = (unsigned)height_blocks(g, fp64 ? 8 : 4);
    if (fp64)
        k_height<double, true, 4, true><<<nb, 256, 0, st>>>(g, (const double *)f, nullptr, h64, zpart,
                                                      maxpart, nullptr, nullptr);
    else
        k_height<float, true, 4, true><<<nb, 256, 0, st>>>(g, (const float *)f, nullptr, h64, zpart,
                                                     maxpart, nullptr, nullptr);
    return hipGetLastError();
}

bool tiling_supported(int lanes, int nv)
{
    if (lanes == kStreamLanes && nv == -kStreamTile) return true;  // streamed rows
#define PDR_SUP(L_, NV_) \
    if (lanes == L_ && nv == NV_) return true;
    PDR_TILINGS(PDR_SUP)
#undef PDR_SUP
    return false;
}

Tiling streamed_tiling() { return Tiling{kStreamLanes, -kStreamTile}; }

int max_tiling_vectors()
{
    int best = 0;
#define PDR_MAXV(L_, NV_) \
    if (L_ * NV_ > best) best = L_ * NV_;
    PDR_TILINGS(PDR_MAXV)
#undef PDR_MAXV
    return best;
}

hipError_t launch_resid(const DevGraph &g, bool fp64, const void *f, const double *h64,
                        const double *Fsum, const double *zpart, int64_t nzpart,
                        const double *maxpart, double *arcpart, double *out, hipStream_t st)
{
    if (g.m > 0) {
        if (fp64)
            k_resid_arc<double><<<g.m, 256, 0, st>>>(g, (const double *)f, h64, Fsum, arcpart);
        else
            k_resid_arc<float><<<g.m, 256, 0, st>>>(g, (const float *)f, h64, Fsum, arcpart);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    k_resid_final<<<1, 1024, 0, st>>>(g, h64, zpart, nzpart, maxpart, arcpart, out);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t count16, hipStream_t st)
{
    k_copy<<<grid_for(count16, 16384), 256, 0, st>>>((const double2 *)src, (double2 *)dst, count16);
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, bool src_fp64, void *dst, bool dst_fp64, int64_t count,
                          hipStream_t st)
{
    const unsigned nb = grid_for(count, 65536);
    if (src_fp64 && dst_fp64)
        k_convert<double, double><<<nb, 256, 0, st>>>((const double *)src, (double *)dst, count);
    else if (src_fp64)
        k_convert<double, float><<<nb, 256, 0, st>>>((const double *)src, (float *)dst, count);
    else if (dst_fp64)
        k_convert<float, double><<<nb, 256, 0, st>>>((const float *)src, (double *)dst, count);
    else
        k_convert<float, float><<<nb, 256, 0, st>>>((const float *)src, (float *)dst, count);
    return hipGetLastError();
}

hipError_t launch_unpad(const DevGraph &g, const void *f, bool f_fp64, void *dst, bool dst_fp64,
                        hipStream_t st)
{
    const unsigned nb = grid_for((int64_t)g.m * g.K, 65536);
    if (f_fp64 && dst_fp64)
        k_unpad<double, double><<<nb, 256, 0, st>>>((const double *)f, (double *)dst, g.m, g.K, g.Kp);
    else if (f_fp64)
        k_unpad<double, float><<<nb, 256, 0, st>>>((const double *)f, (float *)dst, g.m, g.K, g.Kp);
    else if (dst_fp64)
        k_unpad<float, double><<<nb, 256, 0, st>>>((const float *)f, (double *)dst, g.m, g.K, g.Kp);
    else
        k_unpad<float, float><<<nb, 256, 0, st>>>((const float *)f, (float *)dst, g.m, g.K, g.Kp);
    return hipGetLastError();
}

hipError_t launch_pad_rows(const DevGraph &g, const double *src, void *f, bool f_fp64,
                           int64_t row0, int64_t rows, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    const unsigned nb = grid_for(rows * g.Kp, 65536);
    if (f_fp64)
        k_pad<double><<<nb, 256, 0, st>>>(src, (double *)f, row0, rows, g.K, g.Kp);
    else
        k_pad<float><<<nb, 256, 0, st>>>(src, (float *)f, row0, rows, g.K, g.Kp);
    return hipGetLastError();
}

hipError_t launch_pad(const DevGraph &g, const double *src, void *f, bool f_fp64, hipStream_t st)
{
    return launch_pad_rows(g, src, f, f_fp64, 0, g.m, st);
}

// ----------------------------------------------------------------- adjoint (FP64 ESO)
// Reverse mode through PDR-ESO passes (Algorithm 1 with Algorithm 2). Per arc
// the pass map is piecewise linear in c = f + (h_i - h_j)/2: with A the set
// where f' = c - psi/2 > 0, an uncongested arc passes gbar through on A; a
// congested one (psi = (sum_A c - u)/(1 + |A|/2)) gives
// cbar_k = gbar_k - S/(2 + |A|) on A, S = sum_A gbar, and ubar += S/(2 + |A|).
// Through h = Delta/delta and Delta_i = sum_in f - sum_out f + hatDelta_i:
// Dbar_v = (sum_{e out of v} cbar_e - sum_{e into v} cbar_e) / (2 delta_v),
// fbar_e = cbar_e + Dbar_head - Dbar_tail, dbar_k += Dbar_{s_k} - Dbar_{t_k}.

// Seed of the reverse sweep: dz/df = psi_e - (h_i - h_j) on real commodities
// (0 on padding), written as cbar with Dbar = 0 (the form every reverse pass
// reads), and ubar_e = dz/du_e = -psi_e. One item per 16-byte vector of an arc
// row, arcs in the locality order.
__global__ __launch_bounds__(256) void k_adj_seed(DevGraph g, const double *__restrict__ Fsum,
                                                  const double *__restrict__ h,
                                                  double *__restrict__ gbar,
                                                  double *__restrict__ ubar)
{
    const int nvec = g.Kp / 2;
    const int64_t items = (int64_t)g.m * nvec;
    for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < items;
         it += (int64_t)gridDim.x * 256) {
        const int64_t slot = it / nvec;  // arcs in the locality order
        const int q = (int)(it - slot * nvec);
        const int64_t e = g.aorder[slot];
        const double over = Fsum[e] - g.u[e];
        const double psi = over > 0.0 ? over : 0.0;
        const double *hi = h + (int64_t)g.tails[e] * g.Kp;
        const double *hj = h + (int64_t)g.heads[e] * g.Kp;
        double o[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int k = 2 * q + w;
            o[w] = k < g.K ? psi - (hi[k] - hj[k]) : 0.0;
        }
        store_vec(gbar + e * g.Kp + 2 * q, o);
        if (q == 0) ubar[e] = -psi;
    }
}

// dbar_k = dz/dd_k through hatDelta: h_{s_k,k} - h_{t_k,k} (seed, accumulate 0)
// or dbar_k += Dbar_{s_k,k} - Dbar_{t_k,k} (accumulate 1).
__global__ __launch_bounds__(256) void k_adj_dbar(DevGraph g, const double *__restrict__ v,
                                                  double *__restrict__ dbar, int accumulate)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= g.K) return;
    const double x = v[(int64_t)g.s[k] * g.Kp + k] - v[(int64_t)g.t[k] * g.Kp + k];
    dbar[k] = accumulate ? dbar[k] + x : x;
}

// Dbar_v = (sum_out cbar - sum_in cbar) / (2 delta_v), one item per vector of
// a vertex row (out-arcs in CSR order, then in-arcs), vertices in the
// locality order so the two reads of an arc's row fall close together.
__global__ __launch_bounds__(256) void k_adj_vertex(DevGraph g, const double *__restrict__ cbar,
                                                    double *__restrict__ Dbar)
{
    // the height kernel's traversal (commodity-chunk-major items, vertices in
    // locality order, each vertex's incidence list in U = 4 row batches),
    // accumulating sum_in - sum_out of cbar; Dbar = -(that) / (2 delta)
    constexpr int U = 4;
    const int nvec = g.Kp / 2;
    const int64_t Kp = g.Kp;
    const int CV = g.height_cv;
    const int64_t per_chunk = (int64_t)g.n * CV;
    const int64_t total = per_chunk * ((nvec + CV - 1) / CV);
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    for (int64_t gid = blk * 256 + threadIdx.x; gid < total; gid += (int64_t)gridDim.x * 256) {
        const int64_t c = gid / per_chunk;
        const int64_t rem = gid - c * per_chunk;
        const int pos = (int)(rem / CV);
        const int q = (int)(c * CV + (rem - (int64_t)pos * CV));
        if (q >= nvec) continue;
        const int4 vi = *reinterpret_cast<const int4 *>(g.vinfo + 8 * (int64_t)pos);
        const int i = vi.x, p0 = vi.y, pin = vi.y + vi.z, p1 = vi.w;
        const int k0 = 2 * q;
        double acc[2] = {0.0, 0.0};
        for (int p = p0; p < p1; p += U) {
            int e[U];
#pragma unroll
            for (int b = 0; b < U; ++b) e[b] = g.vinc[p + b < p1 ? p + b : p];
            double x[U][2];
#pragma unroll
            for (int b = 0; b < U; ++b) load_vec(cbar + (int64_t)e[b] * Kp + k0, x[b]);
#pragma unroll
            for (int b = 0; b < U; ++b)
                if (p + b < p1) {
                    const double sg = p + b < pin ? 1.0 : -1.0;
                    acc[0] += sg * x[b][0];
                    acc[1] += sg * x[b][1];
                }
        }
        const int dg = p1 - p0;
        double o[2];
        o[0] = dg > 0 ? -acc[0] / (2.0 * dg) : 0.0;
        o[1] = dg > 0 ? -acc[1] / (2.0 * dg) : 0.0;
        store_vec(Dbar + (int64_t)i * Kp + k0, o);
    }
}

hipError_t launch_adj_seed(const DevGraph &g, const double *Fsum, const double *h, double *gbar,
                           double *ubar, double *dbar, hipStream_t st)
{
    if (g.m > 0) {
        k_adj_seed<<<grid_for((int64_t)g.m * (g.Kp / 2), 16384), 256, 0, st>>>(g, Fsum, h, gbar,
                                                                              ubar);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_adj_dbar<<<(g.K + 255) / 256, 256, 0, st>>>(g, h, dbar, 0);
    return hipGetLastError();
}

// The vertex half of a reverse pass: Dbar from the pass's cbar, then dbar.
hipError_t launch_adj_vertex(const DevGraph &g, const double *cbar, double *Dbar, double *dbar,
                             hipStream_t st)
{
    k_adj_vertex<<<(unsigned)height_blocks(g, 8), 256, 0, st>>>(g, cbar, Dbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_adj_dbar<<<(g.K + 255) / 256, 256, 0, st>>>(g, Dbar, dbar, 1);
    return hipGetLastError();
}

// ----------------------------------------------------------------- batched launchers
int arcs_per_block(int lanes) { return lanes > 64 ? 1 : 256 / lanes; }

hipError_t launch_bbegin(const InstView *views, int B, double eps_obj, double z_target,
                         hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    kb_begin<<<(B + 255) / 256, 256, 0, st>>>(views, B, eps_obj, z_target);
    return hipGetLastError();
}

// Number of instances whose stop test has fired, into *out (one block).
__global__ __launch_bounds__(256) void kb_count_stopped(const InstView *__restrict__ views, int B,
                                                        int32_t *__restrict__ out)
{
    __shared__ int part[4];
    int cnt = 0;
    for (int b = threadIdx.x; b < B; b += 256) cnt += views[b].ctrl->stopped ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) *out = part[0] + part[1] + part[2] + part[3];
}

hipError_t launch_bcount_stopped(const InstView *views, int B, int32_t *out, hipStream_t st)
{
    kb_count_stopped<<<1, 256, 0, st>>>(views, B, out);
    return hipGetLastError();
}

hipError_t launch_bheight(const InstView *views, int B, const int2 *hmap, int64_t nblocks,
                          bool fp64, int unroll, hipStream_t st)
{
    if (B <= 0 || nblocks <= 0) return hipSuccess;
    bool launched = false;
#define PDR_BH(U_)                                                                             \
    if (!launched && unroll == U_) {                                                           \
        if (fp64)                                                                              \
            kb_height<double, U_><<<(unsigned)nblocks, 256, 0, st>>>(views, hmap);             \
        else                                                                                   \
            kb_height<float, U_><<<(unsigned)nblocks, 256, 0, st>>>(views, hmap);              \
        launched = true;                                                                       \
    }
    PDR_HEIGHT_UNROLL(PDR_BH)
#undef PDR_BH
    if (!launched) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    kb_reduce<<<B, 1024, 0, st>>>(views);
    return hipGetLastError();
}


}  // namespace pdr
