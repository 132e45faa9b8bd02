// Device code of one PDR sweep for gfx950 (MI355X), shared by the kernel
// translation units (pdr_k_*.hip). Each kernel template here is instantiated
// in exactly one of them.
//
// Data layout in HBM (all row-major, commodity-contiguous, rows padded to Kp):
//   f[e * Kp + k]  pseudo-flow of commodity k on arc e (FP64 or FP32)
//   h[i * Kp + k]  height of commodity k at vertex i (same precision as f)
//   Fsum[e]        FP64 sum over k of the stored f[e, :] (gives psi_e)
// Padded entries (k >= K) are zero and stay zero under both arc updates.
//
// A sweep is three launches on one stream:
//   k_height  excess -> height (Expressions 2-4), one work item per 16-byte
//             vector of a vertex row; FP64 accumulation; per-block partials
//             of sum Delta * h.
//   k_reduce  objective z (Algorithm 1) from those partials and Fsum, the z
//             log, the stop test and the iteration counter (one block).
//   k_eso / k_agd  every arc in parallel (Expression 14 / Algorithm 3). A
//             group of L lanes owns one arc and holds its row in registers;
//             per-arc sums are FP64 group reductions with a fixed tree, so
//             the results do not depend on scheduling.
// No kernel uses atomics; every reduction order is fixed.
#pragma once

#include <limits.h>
#include <math.h>

#include "pdr_internal.h"

namespace pdr {

template <typename T>
struct VecT;
template <>
struct VecT<double> {
    static constexpr int N = 2;
};
template <>
struct VecT<float> {
    static constexpr int N = 4;
};

template <typename T>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&v)[VecT<T>::N])
{
    if constexpr (sizeof(T) == 8) {
        const double2 x = *reinterpret_cast<const double2 *>(p);
        v[0] = x.x;
        v[1] = x.y;
    } else {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    }
}

template <typename T>
__device__ __forceinline__ void store_vec(T *__restrict__ p, const T (&v)[VecT<T>::N])
{
    if constexpr (sizeof(T) == 8) {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    } else {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// Streaming variants for data touched once per kernel (an arc's own flow
// row, a vertex's height row): non-temporal accesses keep such rows from
// evicting the height rows that neighbouring arcs re-read from L2. When a
// pass's whole working set fits in the Infinity Cache the sweep kernels use
// the ordinary forms instead, so the data stays resident between passes
// (DevGraph::temporal).
typedef double pdr_d2 __attribute__((ext_vector_type(2)));
typedef float pdr_f4 __attribute__((ext_vector_type(4)));

template <bool NT, typename T>
__device__ __forceinline__ void load_vec_s(const T *__restrict__ p, T (&v)[VecT<T>::N])
{
    if constexpr (!NT) {
        load_vec(p, v);
    } else if constexpr (sizeof(T) == 8) {
        const pdr_d2 x = __builtin_nontemporal_load(reinterpret_cast<const pdr_d2 *>(p));
        v[0] = x.x;
        v[1] = x.y;
    } else {
        const pdr_f4 x = __builtin_nontemporal_load(reinterpret_cast<const pdr_f4 *>(p));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    }
}

template <bool NT, typename T>
__device__ __forceinline__ void store_vec_s(T *__restrict__ p, const T (&v)[VecT<T>::N])
{
    if constexpr (!NT) {
        store_vec(p, v);
    } else if constexpr (sizeof(T) == 8) {
        pdr_d2 x;
        x.x = v[0];
        x.y = v[1];
        __builtin_nontemporal_store(x, reinterpret_cast<pdr_d2 *>(p));
    } else {
        pdr_f4 x;
        x.x = v[0];
        x.y = v[1];
        x.z = v[2];
        x.w = v[3];
        __builtin_nontemporal_store(x, reinterpret_cast<pdr_f4 *>(p));
    }
}

// Blocks are dispatched round-robin over the 8 XCDs. Remap so that each XCD
// works through one contiguous range of logical blocks; consecutive arcs share
// their tail row of h, which then stays in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    constexpr int64_t NX = 8;
    const int64_t q = nb / NX, r = nb % NX;
    const int64_t x = b % NX, idx = b / NX;
    return x * q + (x < r ? x : r) + idx;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Largest number of values reduced at once by one group_sum call.
constexpr int kRedMax = 4;
// Unit roundoff of FP32.
constexpr double kFp32Unit = 5.9604644775390625e-08;

// Sum of N values over the L lanes of a group; every lane receives the same
// bits (butterfly partners add the same two operands; the cross-wave step
// sums the wave totals in wave order). For L > 64 the group is the whole
// block and `lds` holds 2 * kRedMax * (L / 64) doubles: two halves used
// alternately, so a wave that runs ahead into the next reduction never
// overwrites values another wave is still reading.
template <int L, int N>
__device__ __forceinline__ void group_sum(double (&v)[N], double *lds, int &phase)
{
    static_assert(N <= kRedMax, "too many values in one reduction");
    if constexpr (L == 1) {
        return;
    } else if constexpr (L <= 64) {
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < N; ++q) v[q] += __shfl_xor(v[q], off, L);
    } else {
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
        constexpr int NW = L / 64;
        double *buf = lds + phase * (kRedMax * NW);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int q = 0; q < N; ++q) buf[q * NW + w] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double s = buf[q * NW];
#pragma unroll
            for (int ww = 1; ww < NW; ++ww) s += buf[q * NW + ww];
            v[q] = s;
        }
        phase ^= 1;
    }
}

// ----------------------------------------------------------------- objective + stop test
// One block: z = 1/2 sum of the height kernel's per-block partials of
// Delta * h and of max(0, Fsum_e - u_e)^2 (Algorithm 1), the z log, the stop
// test of Algorithm 1 (|z - z_prev| < eps_obj) or z <= z_target, and the
// iteration counter. The partials come three per height block, so this block
// reads at most 3 * kHeightBlocksMax values. The third is, for FP32 storage,
// z_noise = 1/2 sum_{i,k} (u32 a_ik)^2 / delta_i with a_ik the sum of the
// magnitudes entering Delta_ik and u32 = 2^-24: the objective that rounding
// each stored flow alone would leave; the FP32 run cannot get far below it.
__device__ __forceinline__ void reduce_core(const double *__restrict__ zpart, int nz,
                                            Ctrl *__restrict__ ctrl, double *__restrict__ zlog,
                                            int64_t zmask)
{
    if (ctrl->stopped) return;
    __shared__ double sh[3][16];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = threadIdx.x; q < nz; q += 1024) {
        a += zpart[q];
        b += zpart[nz + q];
        c += zpart[2 * nz + q];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = 0.0, B = 0.0, Cn = 0.0;
        for (int q = 0; q < 16; ++q) {
            A += sh[0][q];
            B += sh[1][q];
            Cn += sh[2][q];
        }
        const double zh = 0.5 * A, zp = 0.5 * B, z = zp + zh;
        ctrl->z_noise = 0.5 * Cn;
        const int64_t ev = ctrl->evals;
        zlog[ev & zmask] = z;
        ctrl->evals = ev + 1;
        ctrl->z = z;
        ctrl->z_psi = zp;
        ctrl->z_h = zh;
        const bool fin = isfinite(z);
        const bool stop = !fin || (ctrl->eps_obj > 0.0 && fabs(z - ctrl->z_prev) < ctrl->eps_obj) ||
                          (ctrl->z_target > 0.0 && z <= ctrl->z_target);
        if (!fin) ctrl->numeric = 1;
        if (stop) {
            ctrl->stopped = 1;
        } else {
            ctrl->z_prev = z;
            ctrl->t_pass = ctrl->t;
            ctrl->t = ctrl->t + 1;
        }
    }
}
// ----------------------------------------------------------------- excess -> height
// Work item (i, q) computes Delta_ik = sum_in f - sum_out f + hatDelta_ik for the
// V commodities of vector q of vertex i, then h = Delta / delta_i. Items are
// visited grid-stride in vertex order, so the two reads of an f row (by its
// tail and by its head) fall close together in time.
// Each block also sums max(0, Fsum_e - u_e)^2 over a grid-stride slice of
// the arcs; zpart[b] and zpart[gridDim + b] receive the two partials.
// RESID: write FP64 heights to h64 and the per-block max |Delta| (residual
// report).
// Work distribution: this block is block `blk` of `nblk` working on g; its
// partials go to slot `part` (zpart[part], zpart[nblk + part], ...).
template <typename T, bool RESID, int U, bool NT = true>
__device__ __forceinline__ void height_core(const DevGraph &g, const T *__restrict__ f,
                                            T *__restrict__ h, double *__restrict__ h64,
                                            double *__restrict__ zpart,
                                            double *__restrict__ maxpart,
                                            const double *__restrict__ Fsum, int64_t blk,
                                            int64_t nblk, int64_t part)
{
    constexpr int V = VecT<T>::N;
    // FP32 storage: also accumulate the size of the rounding noise the stored
    // flows carry into each excess (see k_reduce)
    constexpr bool kNoise = !RESID && sizeof(T) == 4;
    __shared__ double sh[12];
    double ns = 0.0;
    const int nvec = g.Kp / V;
    const int64_t Kp = g.Kp;
    // Items are ordered commodity-chunk-major: chunk c holds vectors
    // [c*CV, (c+1)*CV) of every vertex, vertices in order. All blocks in flight
    // then work on one chunk of a window of consecutive vertices, so the two
    // reads of an arc's chunk (by its tail and by its head) are close in time
    // and the second is served by cache. Blocks are remapped so each XCD walks
    // contiguous vertices (shared in-arc rows stay in that XCD's L2).
    const int CV = g.height_cv;
    const int64_t per_chunk = (int64_t)g.n * CV;
    const int64_t total = per_chunk * ((nvec + CV - 1) / CV);
    double zs = 0.0, mx = 0.0;
    for (int64_t gid = blk * 256 + threadIdx.x; gid < total; gid += nblk * 256) {
        const int64_t c = gid / per_chunk;
        const int64_t rem = gid - c * per_chunk;
        const int pos = (int)(rem / CV);
        const int q = (int)(c * CV + (rem - (int64_t)pos * CV));
        if (q >= nvec) continue;
        // the vertex's record and its incidence list: in-arcs (+) then
        // out-arcs (-), U rows loaded before they are summed (the summation
        // order is the same for every U)
        const int4 vi = *reinterpret_cast<const int4 *>(g.vinfo + 8 * (int64_t)pos);
        // the injection record, loaded with the arc list so its latency
        // overlaps the row loads
        const int4 vj = *reinterpret_cast<const int4 *>(g.vinfo + 8 * (int64_t)pos + 4);
        const int i = vi.x, p0 = vi.y, pin = vi.y + vi.z, p1 = vi.w;
        const int k0 = q * V;
        // mag: the magnitude sum behind the FP32 noise estimate (an estimate,
        // so single precision; it keeps the FP32 kernels within 64 VGPRs)
        double acc[V];
        float mag[V];
#pragma unroll
        for (int w = 0; w < V; ++w) {
            acc[w] = 0.0;
            mag[w] = 0.0f;
        }
        for (int p = p0; p < p1; p += U) {
            int e[U];
#pragma unroll
            for (int b = 0; b < U; ++b) e[b] = g.vinc[p + b < p1 ? p + b : p];
            T x[U][V];
#pragma unroll
            for (int b = 0; b < U; ++b) load_vec(f + (int64_t)e[b] * Kp + k0, x[b]);
#pragma unroll
            for (int b = 0; b < U; ++b)
                if (p + b < p1) {
                    // + for an in-arc, - for an out-arc (sg * x is exact, so
                    // this is acc + x or acc - x rounded once)
                    const double sg = p + b < pin ? 1.0 : -1.0;
#pragma unroll
                    for (int w = 0; w < V; ++w) {
                        acc[w] += sg * (double)x[b][w];
                        if constexpr (kNoise) mag[w] += fabsf((float)x[b][w]);
                    }
                }
        }
        // injections (hatDelta) of this vertex that fall in the vector's
        // commodities [k0, k0 + V): the vertex's list is sorted by commodity,
        // so a binary search finds the first one (a vertex with many
        // commodities would otherwise scan its whole list for every vector)
        if (k0 <= vj.w && k0 + V > vj.z) {
            int lo = vj.x, hi = vj.y;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (g.inj_k[mid] < k0) lo = mid + 1;
                else hi = mid;
            }
            for (int p = lo; p < vj.y && g.inj_k[p] < k0 + V; ++p) {
                const int k = g.inj_k[p] - k0;
                const double val = g.inj_val[p];
#pragma unroll
                for (int w = 0; w < V; ++w)
                    if (w == k) {
                        acc[w] += val;
                        if constexpr (kNoise) mag[w] += (float)fabs(val);
                    }
            }
        }
        const int dg = p1 - p0;
        T hv[V];
        double hd[V];
#pragma unroll
        for (int w = 0; w < V; ++w) {
            const double hh = dg > 0 ? acc[w] / (double)dg : 0.0;
            hd[w] = hh;
            hv[w] = (T)hh;
            zs += acc[w] * hh;
            if (RESID) mx = fmax(mx, fabs(acc[w]));
            if constexpr (kNoise) {
                const double r = kFp32Unit * (double)mag[w];
                if (dg > 0) ns += r * r / (double)dg;
            }
        }
        if constexpr (RESID) {
            double *dst = h64 + (int64_t)i * Kp + k0;
#pragma unroll
            for (int w = 0; w < V; w += 2)
                *reinterpret_cast<double2 *>(dst + w) = make_double2(hd[w], hd[w + 1]);
        } else {
            store_vec_s<NT>(h + (int64_t)i * Kp + k0, hv);
        }
    }
    double ps = 0.0;
    if constexpr (!RESID) {
        for (int64_t e = part * 256 + threadIdx.x; e < g.m; e += nblk * 256) {
            const double over = Fsum[e] - g.u[e];
            if (over > 0.0) ps += over * over;
        }
    }
    zs = wave_sum(zs);
    if (RESID) mx = wave_max(mx);
    else ps = wave_sum(ps);
    if constexpr (kNoise) ns = wave_sum(ns);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = zs;
        sh[4 + w] = RESID ? mx : ps;
        sh[8 + w] = ns;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        zpart[part] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        if (RESID) {
            maxpart[part] = fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
        } else {
            zpart[nblk + part] = (sh[4] + sh[5]) + (sh[6] + sh[7]);
            zpart[2 * nblk + part] = (sh[8] + sh[9]) + (sh[10] + sh[11]);
        }
    }
}

// Eight waves per SIMD (at most 64 VGPRs) for the unrolls up to 4, so that the
// default grid (8 blocks of 4 waves on each of the 256 CUs) is resident at
// once and no block starts late.
template <typename T, bool RESID, int U, bool NT>
__global__ __launch_bounds__(256, (U <= 4 ? 8 : 1)) void k_height(DevGraph g, const T *__restrict__ f,
                                                T *__restrict__ h, double *__restrict__ h64,
                                                double *__restrict__ zpart,
                                                double *__restrict__ maxpart,
                                                const double *__restrict__ Fsum,
                                                const Ctrl *__restrict__ ctrl)
{
    if (!RESID && ctrl->stopped) return;
    height_core<T, RESID, U, NT>(g, f, h, h64, zpart, maxpart, Fsum,
                                 xcd_remap(blockIdx.x, gridDim.x), gridDim.x, blockIdx.x);
}

// ----------------------------------------------------------------- tiled excess -> height
// The vertex-parallel kernel reads each flow row twice, once for each end of
// its arc, and at benchmark sizes the second read mostly misses L2. Here a
// block takes one unit (tile, run of R chunks of kTileVecs vectors) at a time
// and, chunk by chunk, stages that chunk of every arc incident to the tile's
// vertices in LDS, each arc once: an arc with both ends in the tile is read
// from HBM once. Each (vertex, vector) item then sums its incident rows from
// LDS in the order of the vertex-parallel kernel (in-arcs, then out-arcs, by
// ascending id), so the excess and the heights are the same bits.
// Everything that does not depend on the chunk is set up once per unit: the
// row addresses each thread stages, its items' vertex records, the tile's
// slot lists (in LDS) and a cursor into each item's sorted injection list
// (moved forward as the chunks advance). The next chunk's loads are issued
// before the current chunk's sums, so their latency overlaps the LDS work.
// Units run run-major, so tiles sharing an arc stage the same chunks at
// about the same time. LDS: about 39 KiB per block, four blocks per CU.
constexpr int kTileThreads = 256;
constexpr int kTileLoads = (kTileArcs * kTileVecs + kTileThreads - 1) / kTileThreads;
constexpr int kTileItems = (kTileVerts * kTileVecs + kTileThreads - 1) / kTileThreads;
static_assert(kTileThreads % kTileVecs == 0, "a thread keeps one vector slot of every chunk");

template <typename T, bool NT>
__global__ __launch_bounds__(kTileThreads, 4) void k_height_tiled(DevGraph g, int R, const T *__restrict__ f,
                                                        T *__restrict__ h,
                                                        double *__restrict__ zpart,
                                                        const double *__restrict__ Fsum,
                                                        const Ctrl *__restrict__ ctrl)
{
    if (ctrl->stopped) return;
    constexpr int V = VecT<T>::N, CV = kTileVecs, TT = kTileThreads;
    constexpr bool kNoise = sizeof(T) == 4;
    __shared__ __attribute__((aligned(16))) T tile[kTileArcs * CV * V];
    __shared__ uint16_t slots[2 * kTileArcs];
    const int nvec = g.Kp / V;
    const int64_t Kp = g.Kp;
    const int nchunk = (nvec + CV - 1) / CV;
    const int nrun = (nchunk + R - 1) / R;
    const int64_t units = (int64_t)g.ntiles * nrun;
    const int64_t nblk = gridDim.x;
    const int tid = threadIdx.x;
    const int v = tid % CV;  // the vector slot this thread stages and sums in every chunk
    double zs = 0.0, ns = 0.0;
    for (int64_t un = xcd_remap(blockIdx.x, nblk); un < units; un += nblk) {
        const int r = (int)(un / g.ntiles);
        const int t = (int)(un - (int64_t)r * g.ntiles);
        const int4 ti = *reinterpret_cast<const int4 *>(g.tinfo + 4 * (int64_t)t);
        const int nload = (ti.w - ti.z) * CV;
        const int nitem = (ti.y - ti.x) * CV;
        const int P0 = g.vinfo[8 * (int64_t)ti.x + 1];
        const int P1 = g.vinfo[8 * (int64_t)(ti.y - 1) + 3];
        const int c0 = r * R, c1 = min(c0 + R, nchunk);
        for (int p = P0 + tid; p < P1; p += kTileThreads) slots[p - P0] = g.tslot[p];
        int row[kTileLoads];  // arc staged by this thread in load j (-1: none)
#pragma unroll
        for (int j = 0; j < kTileLoads; ++j) {
            const int idx = j * kTileThreads + tid;
            row[j] = idx < nload ? g.tarc[ti.z + idx / CV] : -1;
        }
        int iv[kTileItems], ip0[kTileItems], ipin[kTileItems], ip1[kTileItems];
        int cur[kTileItems], iend[kTileItems], nextk[kTileItems];
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) {
            const int it = k * kTileThreads + tid;
            iv[k] = -1;
            ip0[k] = ipin[k] = ip1[k] = cur[k] = iend[k] = 0;
            nextk[k] = INT_MAX;
            if (it < nitem) {
                const int pos = ti.x + it / CV;
                const int4 vi = *reinterpret_cast<const int4 *>(g.vinfo + 8 * (int64_t)pos);
                const int4 vj = *reinterpret_cast<const int4 *>(g.vinfo + 8 * (int64_t)pos + 4);
                iv[k] = vi.x;
                ip0[k] = vi.y - P0;
                ipin[k] = vi.y + vi.z - P0;
                ip1[k] = vi.w - P0;
                // first injection at or after this item's first commodity
                const int kstart = (c0 * CV + v) * V;
                int lo = vj.x, hi = vj.y;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (g.inj_k[mid] < kstart) lo = mid + 1;
                    else hi = mid;
                }
                cur[k] = lo;
                iend[k] = vj.y;
                nextk[k] = lo < vj.y ? g.inj_k[lo] : INT_MAX;
            }
        }
        auto stage_loads = [&](int c, T (&x)[kTileLoads][V]) {
            const int64_t off = (int64_t)(c * CV + v) * V;
            const bool in = c * CV + v < nvec;
#pragma unroll
            for (int j = 0; j < kTileLoads; ++j) {
                if (row[j] >= 0 && in) {
                    load_vec(f + (int64_t)row[j] * Kp + off, x[j]);
                } else {
#pragma unroll
                    for (int w = 0; w < V; ++w) x[j][w] = (T)0;
                }
            }
        };
        auto put = [&](const T (&x)[kTileLoads][V]) {
#pragma unroll
            for (int j = 0; j < kTileLoads; ++j) {
                const int idx = j * kTileThreads + tid;
                if (idx < nload) store_vec(tile + idx * V, x[j]);
            }
        };
        auto sum_chunk = [&](int c) {
            const int q = c * CV + v;
            if (q >= nvec) return;
            const int k0 = q * V;
#pragma unroll
            for (int k = 0; k < kTileItems; ++k) {
                if (iv[k] < 0) continue;
                double acc[V];
                float mag[V];
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    acc[w] = 0.0;
                    mag[w] = 0.0f;
                }
                // four incident rows read from LDS before they are summed (in
                // order, so the grouping does not change the bits)
                for (int p = ip0[k]; p < ip1[k]; p += 4) {
                    int sl[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) sl[b] = slots[p + b < ip1[k] ? p + b : p];
                    T xv[4][V];
#pragma unroll
                    for (int b = 0; b < 4; ++b) load_vec(tile + (sl[b] * CV + v) * V, xv[b]);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (p + b < ip1[k]) {
                            const double sg = p + b < ipin[k] ? 1.0 : -1.0;
#pragma unroll
                            for (int w = 0; w < V; ++w) {
                                acc[w] += sg * (double)xv[b][w];
                                if constexpr (kNoise) mag[w] += fabsf((float)xv[b][w]);
                            }
                        }
                }
                // injections in [k0, k0 + V); those below k0 belong to other
                // vector slots and are passed over
                while (nextk[k] < k0 + V) {
                    if (nextk[k] >= k0) {
                        const int kk = nextk[k] - k0;
                        const double val = g.inj_val[cur[k]];
#pragma unroll
                        for (int w = 0; w < V; ++w)
                            if (w == kk) {
                                acc[w] += val;
                                if constexpr (kNoise) mag[w] += (float)fabs(val);
                            }
                    }
                    ++cur[k];
                    nextk[k] = cur[k] < iend[k] ? g.inj_k[cur[k]] : INT_MAX;
                }
                const int dg = ip1[k] - ip0[k];
                T hv[V];
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const double hh = dg > 0 ? acc[w] / (double)dg : 0.0;
                    hv[w] = (T)hh;
                    zs += acc[w] * hh;
                    if constexpr (kNoise) {
                        const double rr = kFp32Unit * (double)mag[w];
                        if (dg > 0) ns += rr * rr / (double)dg;
                    }
                }
                store_vec_s<NT>(h + (int64_t)iv[k] * Kp + k0, hv);
            }
        };
        // chunk c + 1 is loaded into registers while chunk c is summed
        T xa[kTileLoads][V];
        stage_loads(c0, xa);
        for (int c = c0; c < c1; ++c) {
            __syncthreads();  // the previous chunk's sums are done with the tile
            put(xa);
            if (c + 1 < c1) stage_loads(c + 1, xa);
            __syncthreads();
            sum_chunk(c);
        }
        __syncthreads();  // the next unit rewrites the slot lists and the tile
    }
    double ps = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kTileThreads + tid; e < g.m; e += nblk * kTileThreads) {
        const double over = Fsum[e] - g.u[e];
        if (over > 0.0) ps += over * over;
    }
    zs = wave_sum(zs);
    ps = wave_sum(ps);
    if constexpr (kNoise) ns = wave_sum(ns);
    // the staging area is free here (every unit ended with a barrier)
    constexpr int NW = TT / 64;
    double *sh = reinterpret_cast<double *>(tile);
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        sh[w] = zs;
        sh[NW + w] = ps;
        sh[2 * NW + w] = ns;
    }
    __syncthreads();
    if (tid == 0) {
        double a = sh[0], b = sh[NW], cc = sh[2 * NW];
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            a += sh[q];
            b += sh[NW + q];
            cc += sh[2 * NW + q];
        }
        const int64_t part = blockIdx.x;
        zpart[part] = a;
        zpart[nblk + part] = b;
        zpart[2 * nblk + part] = cc;
    }
}

// Batched: hmap[logical block] = (instance, block within the instance); the
// blocks of one instance are consecutive logical blocks, so an instance stays
// on one XCD's range.
template <typename T, int U>
__global__ __launch_bounds__(256) void kb_height(const InstView *__restrict__ views,
                                                 const int2 *__restrict__ hmap)
{
    const int2 it = hmap[xcd_remap(blockIdx.x, gridDim.x)];
    const InstView &I = views[it.x];
    if (I.ctrl->stopped) return;
    height_core<T, false, U>(I.g, (const T *)I.f, (T *)I.h, nullptr, I.zpart, nullptr, I.Fsum,
                             it.y, I.nzpart, it.y);
}
// ----------------------------------------------------------------- arc kernels
template <int L>
struct ArcShape {
    static constexpr int BS = L > 64 ? L : 256;  // block size
    static constexpr int GPB = BS / L;           // arcs per block
    static constexpr int NW = L > 64 ? L / 64 : 1;
};

// PDR-ESO arc update: the exact minimiser of the edge subproblem
// (Expression 14). With c_k = ((h_ik + f_k) - (h_jk - f_k)) / 2 (Algorithm 2),
// the new flows are f'_k = max(0, c_k - psi/2) where psi = 0 if
// sum_k max(0, c_k) <= u, and otherwise psi is the root of
// psi = sum_k max(0, c_k - psi/2) - u. The root is found without sorting by
// the finite active-set iteration of Michelot (1986) for projections onto a
// simplex: with A = {k: c_k > 0}, repeat psi = (sum_A c - u) / (1 + |A|/2),
// A <- {k in A: c_k > psi/2} until A is unchanged. Each pass is one group
// reduction of (sum, count) over the register-resident c.
// CAP: the capacity-enforcing step of Section 6's formulation instead (no
// congestion term, sum f' <= u kept): f'_k = max(0, c_k - lambda), the
// projection of c onto {f >= 0, sum f <= u}, with lambda = (sum_A c - u)/|A|
// found by the same iteration; at u = 0 the set can empty (every c equal to
// lambda), which also ends it.
// fin: the flows to read when they differ from the flows written (f), as in
// the adjoint's recomputation of a segment; nullptr updates f in place.
template <typename T, int L, int NV, bool CAP = false, bool NT = true>
__device__ __forceinline__ void eso_arc(const DevGraph &g, T *__restrict__ f, const T *__restrict__ h, double *__restrict__ Fsum, int64_t slot, int lane, double *lds, const T *__restrict__ fin = nullptr)
{
    constexpr int V = VecT<T>::N;
    int phase = 0;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    const T *fe = (fin ? fin : f) + e * Kp;
    const T *hi = h + (int64_t)g.tails[e] * Kp;
    const T *hj = h + (int64_t)g.heads[e] * Kp;
    const double u = g.u[e];

    // The lane's f vectors are all requested before the first is used, so the
    // whole row is in flight at once (a lane past the row's end re-reads its
    // last vector, which stays in bounds, and keeps c = 0); the h rows, mostly
    // cache hits, follow one vector at a time.
    T c[NV][V];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        load_vec_s<NT>(fe + (q < nvec ? q : nvec - 1) * V, c[v]);
    }
    double red[2] = {0.0, 0.0};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            T a[V], b[V];
            load_vec(hi + q * V, a);
            load_vec(hj + q * V, b);
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const T x = c[v][w];
                const T cc = (T)0.5 * ((a[w] + x) - (b[w] - x));
                c[v][w] = cc;
                if (cc > (T)0) {
                    red[0] += (double)cc;
                    red[1] += 1.0;
                }
            }
        } else {
#pragma unroll
            for (int w = 0; w < V; ++w) c[v][w] = (T)0;
        }
    }
    group_sum<L, 2>(red, lds, phase);
    double Ssum = red[0], P = red[1];
    double half = 0.0;  // psi/2 (ESO) or lambda (CAP): the shift of the active c
    // Without congestion the new row is max(0, c): its terms, and their
    // summation order, are those of the reduction above, so its sum is Ssum
    // exactly and the group (which ends with this arc) needs no second
    // reduction.
    const bool congested = Ssum > u;
    if (!congested) {
        if (lane == 0) Fsum[e] = Ssum;
    } else {
        double theta = 0.0;
        for (;;) {
            half = CAP ? (Ssum - u) / P : 0.5 * ((Ssum - u) / (1.0 + 0.5 * P));
            const double th = fmax(theta, half);
            double r2[2] = {0.0, 0.0};
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const double cc = (double)c[v][w];
                    if (cc > th) {
                        r2[0] += cc;
                        r2[1] += 1.0;
                    }
                }
            group_sum<L, 2>(r2, lds, phase);
            // active set unchanged: the shift is the root
            if (r2[1] == P || (CAP && r2[1] == 0.0)) break;
            Ssum = r2[0];
            P = r2[1];
            theta = th;
        }
    }
    double fs[1] = {0.0};
    T *fo = f + e * Kp;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            T o[V];
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const double val = (double)c[v][w] - half;
                o[w] = (T)(val > 0.0 ? val : 0.0);
                fs[0] += (double)o[w];
            }
            store_vec_s<NT>(fo + q * V, o);
        }
    }
    if (congested) {
        group_sum<L, 1>(fs, lds, phase);
        if (lane == 0) Fsum[e] = fs[0];
    }
}

template <typename T, int L, int NV, bool CAP, bool NT>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_eso(DevGraph g, T *__restrict__ f,
                                                          const T *__restrict__ h,
                                                          double *__restrict__ Fsum,
                                                          const Ctrl *__restrict__ ctrl)
{
    if (ctrl->stopped) return;
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    eso_arc<T, L, NV, CAP, NT>(g, f, h, Fsum, slot, lane, lds);
}

// One FP64 PDR-ESO pass out of place: reads fin, writes fout (the adjoint
// recomputes a segment's flows from a checkpoint without copying it first).
template <int L, int NV>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_eso_oop(DevGraph g,
                                                              const double *__restrict__ fin,
                                                              double *__restrict__ fout,
                                                              const double *__restrict__ h,
                                                              double *__restrict__ Fsum)
{
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    eso_arc<double, L, NV, false, true>(g, fout, h, Fsum, slot, lane, lds, fin);
}

// Batched: amap[logical block] = (instance, block within the instance's arcs).
template <typename T, int L, int NV, bool CAP>
__global__ __launch_bounds__(ArcShape<L>::BS) void kb_eso(const InstView *__restrict__ views,
                                                          const int2 *__restrict__ amap)
{
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int2 it = amap[xcd_remap(blockIdx.x, gridDim.x)];
    const InstView &I = views[it.x];
    if (I.ctrl->stopped) return;
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = (int64_t)it.y * S::GPB + grp;
    if (L <= 64 && slot >= I.g.m) return;
    eso_arc<T, L, NV, CAP>(I.g, (T *)I.f, (const T *)I.h, I.Fsum, slot, lane, lds);
}

// PDR-AGD arc update (Algorithm 3): phi_k = h_ik - h_jk - psi,
// df_k = max(-f_k, beta phi_k); the step is kept iff the exact change of the
// edge subproblem objective (Expression 13, optimal slack),
// dz = 1/2[(F + sum df - u)_+^2 - psi^2] + sum_k df_k (df_k - (h_ik - h_jk)),
// is <= 0; otherwise beta <- max(beta_min, alpha_dec beta). Every inc_period
// iterations beta <- min(beta_max, alpha_inc beta).
template <typename T, int L, int NV, bool NT = true, bool RowFirst = false>
__device__ __forceinline__ void agd_arc(const DevGraph &g, T *__restrict__ f, const T *__restrict__ h, double *__restrict__ Fsum, double *__restrict__ beta, const AgdParams &prm, const Ctrl *__restrict__ ctrl, int64_t slot, int lane, double *lds)
{
    constexpr int V = VecT<T>::N;
    int phase = 0;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    const T *fe = f + e * Kp;
    const T *hi = h + (int64_t)g.tails[e] * Kp;
    const T *hj = h + (int64_t)g.heads[e] * Kp;
    const double u = g.u[e];
    const double F = Fsum[e];
    const double psi = F > u ? F - u : 0.0;
    const double b = beta[e];

    // the stepped row f + df, written only if the step is accepted; it first
    // holds the row itself. RowFirst: all of a lane's f vectors are requested
    // before the first is used (a lane past the row's end re-reads its last
    // vector); otherwise they are loaded one vector at a time, which needs
    // fewer registers. The single-instance AGD kernel takes RowFirst with 512
    // or more lanes per arc, where it leaves the occupancy unchanged.
    constexpr bool kRowFirst = RowFirst;
    T cand[NV][V];
    if constexpr (kRowFirst) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int q = v * L + lane;
            load_vec_s<NT>(fe + (q < nvec ? q : nvec - 1) * V, cand[v]);
        }
    }
    double red[3] = {0.0, 0.0, 0.0};  // sum df, sum df (df - g), sum of stepped values
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            T a[V], bb[V];
            if constexpr (!kRowFirst) load_vec_s<NT>(fe + q * V, cand[v]);
            load_vec(hi + q * V, a);
            load_vec(hj + q * V, bb);
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const double gg = (double)(a[w] - bb[w]);
                const double fx = (double)cand[v][w];
                const double step = b * (gg - psi);
                const double df = step > -fx ? step : -fx;
                cand[v][w] = (T)(fx + df);
                red[0] += df;
                red[1] += df * (df - gg);
                red[2] += (double)cand[v][w];
            }
        } else {
#pragma unroll
            for (int w = 0; w < V; ++w) cand[v][w] = (T)0;
        }
    }
    group_sum<L, 3>(red, lds, phase);
    // congestion part 1/2[(F + S - u)_+^2 - (F - u)_+^2]; factored as
    // S (F - u + S/2) when over capacity before and after the step, so that a
    // small step is not lost in the difference of two large squares
    const double before = F - u, after = F + red[0] - u;
    const double dcong = (before > 0.0 && after > 0.0)
                             ? red[0] * (before + 0.5 * red[0])
                             : 0.5 * ((after > 0.0 ? after * after : 0.0) -
                                      (before > 0.0 ? before * before : 0.0));
    const double dz = dcong + red[1];
    const bool accept = dz <= 0.0;
    if (accept) {
        T *fo = f + e * Kp;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int q = v * L + lane;
            if (q < nvec) store_vec_s<NT>(fo + q * V, cand[v]);
        }
    }
    if (lane == 0) {
        double nb = b;
        if (!accept) nb = fmax(prm.beta_min, nb * prm.alpha_dec);
        if (prm.inc_period > 0 && (ctrl->t_pass % prm.inc_period) == 0)
            nb = fmin(prm.beta_max, nb * prm.alpha_inc);
        beta[e] = nb;
        if (accept) Fsum[e] = red[2];
    }
}

template <typename T, int L, int NV, bool NT>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_agd(DevGraph g, T *__restrict__ f,
                                                          const T *__restrict__ h,
                                                          double *__restrict__ Fsum,
                                                          double *__restrict__ beta,
                                                          AgdParams prm,
                                                          const Ctrl *__restrict__ ctrl)
{
    if (ctrl->stopped) return;
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    agd_arc<T, L, NV, NT, (L >= 512)>(g, f, h, Fsum, beta, prm, ctrl, slot, lane, lds);
}

// Batched: amap[logical block] = (instance, block within the instance's arcs).
template <typename T, int L, int NV>
__global__ __launch_bounds__(ArcShape<L>::BS) void kb_agd(const InstView *__restrict__ views,
                                                          const int2 *__restrict__ amap)
{
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int2 it = amap[xcd_remap(blockIdx.x, gridDim.x)];
    const InstView &I = views[it.x];
    if (I.ctrl->stopped) return;
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = (int64_t)it.y * S::GPB + grp;
    if (L <= 64 && slot >= I.g.m) return;
    agd_arc<T, L, NV>(I.g, (T *)I.f, (const T *)I.h, I.Fsum, I.beta, I.prm, I.ctrl, slot, lane, lds);
}

// PDR-GDM arc update (Algorithm 4): the step df and its accept test are those
// of Algorithm 3 (k_agd); an accepted arc takes v' = gamma v + df and
// f' = max(0, f + v'), a rejected one keeps f and v and lowers beta. beta's
// periodic increase is as in k_agd.
template <typename T, int L, int NV, bool NT = true>
__device__ __forceinline__ void gdm_arc(const DevGraph &g, T *__restrict__ f, T *__restrict__ vel, const T *__restrict__ h, double *__restrict__ Fsum, double *__restrict__ beta, const AgdParams &prm, const Ctrl *__restrict__ ctrl, int64_t slot, int lane, double *lds)
{
    constexpr int V = VecT<T>::N;
    int phase = 0;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    const T *fe = f + e * Kp;
    const T *ve = vel + e * Kp;
    const T *hi = h + (int64_t)g.tails[e] * Kp;
    const T *hj = h + (int64_t)g.heads[e] * Kp;
    const double u = g.u[e];
    const double F = Fsum[e];
    const double psi = F > u ? F - u : 0.0;
    const double b = beta[e];
    const double gam = prm.gamma;

    T nf[NV][V], nv[NV][V];  // the row's new flows and velocities if accepted
    double red[3] = {0.0, 0.0, 0.0};  // sum df, sum df (df - g), sum of new flows
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            T a[V], bb[V], x[V], w0[V];
            load_vec_s<NT>(fe + q * V, x);
            load_vec_s<NT>(ve + q * V, w0);
            load_vec(hi + q * V, a);
            load_vec(hj + q * V, bb);
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const double gg = (double)(a[w] - bb[w]);
                const double fx = (double)x[w];
                const double step = b * (gg - psi);
                const double df = step > -fx ? step : -fx;
                const double vn = gam * (double)w0[w] + df;
                const double fn = fx + vn;
                nv[v][w] = (T)vn;
                nf[v][w] = (T)(fn > 0.0 ? fn : 0.0);
                red[0] += df;
                red[1] += df * (df - gg);
                red[2] += (double)nf[v][w];
            }
        } else {
#pragma unroll
            for (int w = 0; w < V; ++w) nf[v][w] = nv[v][w] = (T)0;
        }
    }
    group_sum<L, 3>(red, lds, phase);
    const double before = F - u, after = F + red[0] - u;
    const double dcong = (before > 0.0 && after > 0.0)
                             ? red[0] * (before + 0.5 * red[0])
                             : 0.5 * ((after > 0.0 ? after * after : 0.0) -
                                      (before > 0.0 ? before * before : 0.0));
    const bool accept = dcong + red[1] <= 0.0;
    if (accept) {
        T *fo = f + e * Kp;
        T *vo = vel + e * Kp;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int q = v * L + lane;
            if (q < nvec) {
                store_vec_s<NT>(fo + q * V, nf[v]);
                store_vec_s<NT>(vo + q * V, nv[v]);
            }
        }
    }
    if (lane == 0) {
        double nb = b;
        if (!accept) nb = fmax(prm.beta_min, nb * prm.alpha_dec);
        if (prm.inc_period > 0 && (ctrl->t_pass % prm.inc_period) == 0)
            nb = fmin(prm.beta_max, nb * prm.alpha_inc);
        beta[e] = nb;
        if (accept) Fsum[e] = red[2];
    }
}

template <typename T, int L, int NV, bool NT>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_gdm(DevGraph g, T *__restrict__ f,
                                                          T *__restrict__ vel,
                                                          const T *__restrict__ h,
                                                          double *__restrict__ Fsum,
                                                          double *__restrict__ beta,
                                                          AgdParams prm,
                                                          const Ctrl *__restrict__ ctrl)
{
    if (ctrl->stopped) return;
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    gdm_arc<T, L, NV, NT>(g, f, vel, h, Fsum, beta, prm, ctrl, slot, lane, lds);
}

// Batched: amap[logical block] = (instance, block within the instance's arcs).
template <typename T, int L, int NV>
__global__ __launch_bounds__(ArcShape<L>::BS) void kb_gdm(const InstView *__restrict__ views,
                                                          const int2 *__restrict__ amap)
{
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int2 it = amap[xcd_remap(blockIdx.x, gridDim.x)];
    const InstView &I = views[it.x];
    if (I.ctrl->stopped) return;
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = (int64_t)it.y * S::GPB + grp;
    if (L <= 64 && slot >= I.g.m) return;
    gdm_arc<T, L, NV>(I.g, (T *)I.f, (T *)I.v, (const T *)I.h, I.Fsum, I.beta, I.prm, I.ctrl, slot, lane, lds);
}

// Fsum[e] = sum_k f[e, k] with the same lane layout and reduction tree as the
// arc kernels (so a restored state continues bit for bit).
template <typename T, int L, int NV>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_rowsum(DevGraph g, const T *__restrict__ f,
                                                             double *__restrict__ Fsum)
{
    constexpr int V = VecT<T>::N;
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    int phase = 0;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    const int64_t e = g.aorder[slot];
    const int nvec = g.Kp / V;
    const T *fe = f + e * (int64_t)g.Kp;
    double fs[1] = {0.0};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            T x[V];
            load_vec_s<true>(fe + q * V, x);
#pragma unroll
            for (int w = 0; w < V; ++w) fs[0] += (double)x[w];
        }
    }
    group_sum<L, 1>(fs, lds, phase);
    if (lane == 0) Fsum[e] = fs[0];
}

// ----------------------------------------------------------------- long rows
// Rows longer than the register-resident arc kernels hold (more than
// max_tiling_vectors() 16-byte vectors): one block of kStreamLanes lanes per
// arc streams the row in tiles of kStreamLanes x TV vectors, with the same
// per-element arithmetic as the resident kernels. PDR-ESO needs one pass
// (reading f, h_i, h_j and writing max(0, c) in place) for an arc within
// capacity, and for a congested one also a pass over its own row per step of
// the threshold iteration and one for the update; PDR-AGD and PDR-GDM one
// pass that stores the stepped row in place (and a second that restores it
// if the step is rejected). Stores are streaming.
constexpr int kStreamLanes = 1024;
// vectors per lane of one tile; Tiling{kStreamLanes, -kStreamTile} names the
// streamed arc kernels
constexpr int kStreamTile = 4;

// The TV vectors of lane `lane` in the tile at `base` of a streamed row, all
// requested before any is used (a lane past the row's end re-reads its last
// vector, which stays in bounds; callers skip it).
template <typename T, int TV>
__device__ __forceinline__ void load_tile(const T *__restrict__ p, int base, int lane, int nvec,
                                          T (&x)[TV][VecT<T>::N])
{
    constexpr int V = VecT<T>::N;
#pragma unroll
    for (int v = 0; v < TV; ++v) {
        const int q = base + v * kStreamLanes + lane;
        load_vec(p + (q < nvec ? q : nvec - 1) * V, x[v]);
    }
}

// The first pass also stores max(c, 0) in place of the row. Every later step
// needs only that: the threshold th = max(theta, half) is never negative, so
// c > th exactly where the stored value exceeds th, and max(c - half, 0) equals
// max(stored - half, 0) (an entry with c <= 0 ends at zero either way). An
// arc whose positive sum stays within its capacity (half = 0) is then done
// after one pass; a congested one re-reads only its own row.
template <typename T, int TV, bool CAP>
__device__ __forceinline__ void eso_arc_stream(const DevGraph &g, T *__restrict__ f,
                                               const T *__restrict__ h, double *__restrict__ Fsum,
                                               int64_t slot, int lane, double *lds)
{
    constexpr int L = kStreamLanes, V = VecT<T>::N;
    int phase = 0;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    T *fe = f + e * Kp;
    const T *hi = h + (int64_t)g.tails[e] * Kp;
    const T *hj = h + (int64_t)g.heads[e] * Kp;
    const double u = g.u[e];
    double red[2] = {0.0, 0.0};
    for (int base = 0; base < nvec; base += L * TV) {
        T x[TV][V];
        load_tile<T, TV>(fe, base, lane, nvec, x);
#pragma unroll
        for (int v = 0; v < TV; ++v) {
            const int q = base + v * L + lane;
            if (q < nvec) {
                T a[V], b[V], o[V];
                load_vec(hi + q * V, a);
                load_vec(hj + q * V, b);
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const T c = (T)0.5 * ((a[w] + x[v][w]) - (b[w] - x[v][w]));
                    o[w] = c > (T)0 ? c : (T)0;
                    if (c > (T)0) {
                        red[0] += (double)c;
                        red[1] += 1.0;
                    }
                }
                store_vec_s<true>(fe + q * V, o);
            }
        }
    }
    group_sum<L, 2>(red, lds, phase);
    double Ssum = red[0], P = red[1];
    if (Ssum <= u) {
        // half = 0: the stored row is the new row and its sum is Ssum (the
        // same terms summed in the same order)
        if (lane == 0) Fsum[e] = Ssum;
        return;
    }
    double half = 0.0;
    double theta = 0.0;
    for (;;) {
        half = CAP ? (Ssum - u) / P : 0.5 * ((Ssum - u) / (1.0 + 0.5 * P));
        const double th = fmax(theta, half);
        double r2[2] = {0.0, 0.0};
        for (int base = 0; base < nvec; base += L * TV) {
            T x[TV][V];
            load_tile<T, TV>(fe, base, lane, nvec, x);
#pragma unroll
            for (int v = 0; v < TV; ++v) {
                const int q = base + v * L + lane;
                if (q < nvec) {
#pragma unroll
                    for (int w = 0; w < V; ++w) {
                        const double cc = (double)x[v][w];
                        if (cc > th) {
                            r2[0] += cc;
                            r2[1] += 1.0;
                        }
                    }
                }
            }
        }
        group_sum<L, 2>(r2, lds, phase);
        if (r2[1] == P || (CAP && r2[1] == 0.0)) break;
        Ssum = r2[0];
        P = r2[1];
        theta = th;
    }
    double fs[1] = {0.0};
    for (int base = 0; base < nvec; base += L * TV) {
        T x[TV][V];
        load_tile<T, TV>(fe, base, lane, nvec, x);
#pragma unroll
        for (int v = 0; v < TV; ++v) {
            const int q = base + v * L + lane;
            if (q < nvec) {
                T o[V];
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const double val = (double)x[v][w] - half;
                    o[w] = (T)(val > 0.0 ? val : 0.0);
                    fs[0] += (double)o[w];
                }
                store_vec_s<true>(fe + q * V, o);
            }
        }
    }
    group_sum<L, 1>(fs, lds, phase);
    if (lane == 0) Fsum[e] = fs[0];
}

template <typename T, int TV, bool CAP>
__global__ __launch_bounds__(kStreamLanes) void k_eso_stream(DevGraph g, T *__restrict__ f,
                                                             const T *__restrict__ h,
                                                             double *__restrict__ Fsum,
                                                             const Ctrl *__restrict__ ctrl)
{
    if (ctrl->stopped) return;
    __shared__ double lds[2 * kRedMax * (kStreamLanes / 64)];
    eso_arc_stream<T, TV, CAP>(g, f, h, Fsum, xcd_remap(blockIdx.x, gridDim.x), (int)threadIdx.x,
                               lds);
}

// AGD (vel == nullptr) or GDM arc step on a streamed row, in one pass over
// it: each vector's stepped values (new flows, and velocities) are stored in
// place at once, its old values in the block's undo rows (uf, uv), while the
// sums of df, df (df - g) and the new values are formed; a rejected step then
// copies the old values back. An accepted step (the common case: the rate
// falls on a rejection and grows only every inc_period passes) so reads the
// row, h_i and h_j once instead of twice.
template <typename T, int TV, bool GDM>
__device__ __forceinline__ void agd_arc_stream(const DevGraph &g, T *__restrict__ f,
                                               T *__restrict__ vel, const T *__restrict__ h,
                                               double *__restrict__ Fsum, double *__restrict__ beta,
                                               const AgdParams &prm, const Ctrl *__restrict__ ctrl,
                                               int64_t slot, int lane, double *lds, int &phase,
                                               T *__restrict__ uf, T *__restrict__ uv)
{
    constexpr int L = kStreamLanes, V = VecT<T>::N;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    T *fe = f + e * Kp;
    T *ve = GDM ? vel + e * Kp : nullptr;
    const T *hi = h + (int64_t)g.tails[e] * Kp;
    const T *hj = h + (int64_t)g.heads[e] * Kp;
    const double u = g.u[e];
    const double F = Fsum[e];
    const double psi = F > u ? F - u : 0.0;
    const double b = beta[e];
    const double gam = prm.gamma;
    double red[3] = {0.0, 0.0, 0.0};  // sum df, sum df (df - g), sum of the new values
    for (int base = 0; base < nvec; base += L * TV) {
        T x[TV][V], w0[TV][V];
        load_tile<T, TV>(fe, base, lane, nvec, x);
        if constexpr (GDM) load_tile<T, TV>(ve, base, lane, nvec, w0);
#pragma unroll
        for (int v = 0; v < TV; ++v) {
            const int q = base + v * L + lane;
            if (q < nvec) {
                T a[V], bb[V], nf[V], nv[V];
                load_vec(hi + q * V, a);
                load_vec(hj + q * V, bb);
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const double gg = (double)(a[w] - bb[w]);
                    const double fx = (double)x[v][w];
                    const double st = b * (gg - psi);
                    const double df = st > -fx ? st : -fx;
                    if constexpr (GDM) {
                        const double vn = gam * (double)w0[v][w] + df;
                        const double fn = fx + vn;
                        nv[w] = (T)vn;
                        nf[w] = (T)(fn > 0.0 ? fn : 0.0);
                    } else {
                        nf[w] = (T)(fx + df);
                    }
                    red[0] += df;
                    red[1] += df * (df - gg);
                    red[2] += (double)nf[w];
                }
                store_vec_s<true>(uf + q * V, x[v]);
                store_vec_s<true>(fe + q * V, nf);
                if constexpr (GDM) {
                    store_vec_s<true>(uv + q * V, w0[v]);
                    store_vec_s<true>(ve + q * V, nv);
                }
            }
        }
    }
    group_sum<L, 3>(red, lds, phase);
    const double before = F - u, after = F + red[0] - u;
    const double dcong = (before > 0.0 && after > 0.0)
                             ? red[0] * (before + 0.5 * red[0])
                             : 0.5 * ((after > 0.0 ? after * after : 0.0) -
                                      (before > 0.0 ? before * before : 0.0));
    const bool accept = dcong + red[1] <= 0.0;
    if (!accept) {
        // each lane restores the vectors it wrote itself
        for (int base = 0; base < nvec; base += L * TV)
#pragma unroll
            for (int v = 0; v < TV; ++v) {
                const int q = base + v * L + lane;
                if (q < nvec) {
                    T x[V];
                    load_vec(uf + q * V, x);
                    store_vec_s<true>(fe + q * V, x);
                    if constexpr (GDM) {
                        T w0[V];
                        load_vec(uv + q * V, w0);
                        store_vec_s<true>(ve + q * V, w0);
                    }
                }
            }
    }
    if (lane == 0) {
        double nb = b;
        if (!accept) nb = fmax(prm.beta_min, nb * prm.alpha_dec);
        if (prm.inc_period > 0 && (ctrl->t_pass % prm.inc_period) == 0)
            nb = fmin(prm.beta_max, nb * prm.alpha_inc);
        beta[e] = nb;
        if (accept) Fsum[e] = red[2];
    }
}

// The streamed AGD / GDM kernels run kStreamSlots blocks (one per CU, as their
// registers allow) in a grid-stride loop over the arcs, each block with its
// own undo rows.
template <typename T, int TV, bool GDM>
__global__ __launch_bounds__(kStreamLanes) void k_agd_stream(DevGraph g, T *__restrict__ f,
                                                             T *__restrict__ vel,
                                                             const T *__restrict__ h,
                                                             double *__restrict__ Fsum,
                                                             double *__restrict__ beta,
                                                             AgdParams prm,
                                                             const Ctrl *__restrict__ ctrl,
                                                             T *__restrict__ undo)
{
    if (ctrl->stopped) return;
    __shared__ double lds[2 * kRedMax * (kStreamLanes / 64)];
    const int64_t Kp = g.Kp;
    T *uf = undo + (int64_t)blockIdx.x * (GDM ? 2 : 1) * Kp;
    T *uv = GDM ? uf + Kp : nullptr;
    const int64_t nblk = gridDim.x;
    // the reduction buffer's halves alternate across the block's arcs too, so
    // a wave that runs ahead into the next arc's reduction cannot overwrite
    // values a slower wave is still reading
    int phase = 0;
    for (int64_t s = xcd_remap(blockIdx.x, nblk); s < g.m; s += nblk)
        agd_arc_stream<T, TV, GDM>(g, f, vel, h, Fsum, beta, prm, ctrl, s, (int)threadIdx.x, lds,
                                   phase, uf, uv);
}

// Fsum of a streamed row.
template <typename T, int TV>
__global__ __launch_bounds__(kStreamLanes) void k_rowsum_stream(DevGraph g,
                                                                const T *__restrict__ f,
                                                                double *__restrict__ Fsum)
{
    constexpr int V = VecT<T>::N, L = kStreamLanes;
    __shared__ double lds[2 * kRedMax * (L / 64)];
    int phase = 0;
    const int64_t e = g.aorder[xcd_remap(blockIdx.x, gridDim.x)];
    const int nvec = g.Kp / V;
    const T *fe = f + e * (int64_t)g.Kp;
    double fs[1] = {0.0};
    const int lane = (int)threadIdx.x;
    for (int base = 0; base < nvec; base += L * TV)
#pragma unroll
        for (int v = 0; v < TV; ++v) {
            const int q = base + v * L + lane;
            if (q < nvec) {
                T x[V];
                load_vec(fe + q * V, x);
#pragma unroll
                for (int w = 0; w < V; ++w) fs[0] += (double)x[w];
            }
        }
    group_sum<L, 1>(fs, lds, phase);
    if (lane == 0) Fsum[e] = fs[0];
}

// ----------------------------------------------------------------- residual report
// Per arc: sum_k rho_k^2 (rho = phi if f > 0 else max(0, phi)), u_e l_e with
// l_e = max(0, max_k (h_ik - h_jk)), and psi_e. One block per arc.
template <typename T>
__global__ __launch_bounds__(256) void k_resid_arc(DevGraph g, const T *__restrict__ f,
                                                   const double *__restrict__ h64,
                                                   const double *__restrict__ Fsum,
                                                   double *__restrict__ arcpart)
{
    __shared__ double sh[8];
    const int e = blockIdx.x;
    const int64_t Kp = g.Kp;
    const double *hi = h64 + (int64_t)g.tails[e] * Kp;
    const double *hj = h64 + (int64_t)g.heads[e] * Kp;
    const T *fe = f + (int64_t)e * Kp;
    const double u = g.u[e];
    const double F = Fsum[e];
    const double psi = F > u ? F - u : 0.0;
    double kkt = 0.0, lmax = 0.0;
    for (int k = threadIdx.x; k < g.K; k += 256) {
        const double gg = hi[k] - hj[k];
        const double phi = gg - psi;
        const double rho = (double)fe[k] > 0.0 ? phi : (phi > 0.0 ? phi : 0.0);
        kkt += rho * rho;
        lmax = fmax(lmax, gg);
    }
    kkt = wave_sum(kkt);
    lmax = wave_max(lmax);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = kkt;
        sh[4 + w] = lmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        arcpart[e] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        arcpart[g.m + e] = u * fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
        arcpart[2 * (int64_t)g.m + e] = psi;
    }
}

// ----------------------------------------------------------------- copies
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(const S *__restrict__ src, D *__restrict__ dst,
                                                 int64_t count)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * 256)
        dst[q] = (D)src[q];
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void k_unpad(const S *__restrict__ f, D *__restrict__ dst,
                                               int64_t m, int K, int Kp)
{
    const int64_t total = m * (int64_t)K;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * 256) {
        const int64_t e = q / K;
        const int k = (int)(q - e * K);
        dst[q] = (D)f[e * Kp + k];
    }
}

// Rows [row0, row0 + rows) of f from src, which holds those rows unpadded
// (src[(e - row0) * K + k]).
template <typename D>
__global__ __launch_bounds__(256) void k_pad(const double *__restrict__ src, D *__restrict__ f,
                                             int64_t row0, int64_t rows, int K, int Kp)
{
    const int64_t total = rows * (int64_t)Kp;
    D *dst = f + row0 * (int64_t)Kp;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * 256) {
        const int64_t e = q / Kp;
        const int k = (int)(q - e * Kp);
        dst[q] = k < K ? (D)src[e * K + k] : (D)0;
    }
}

// ----------------------------------------------------------------- adjoint arc pass (FP64 ESO)
// ESO pass, reverse: from f^t, h^t and dz/df^(t+1) = cbar + Dbar_head -
// Dbar_tail (the previous reverse pass's outputs, or the seed with Dbar = 0),
// the pass's cbar (written over the arc's own cbar row: each lane rewrites
// only the elements it read) and ubar += S/(2 + |A|). c and psi are recomputed
// with the forward kernel's arithmetic and reduction tree (same tiling), so A
// is the forward pass's set.
template <int L, int NV>
__device__ __forceinline__ void eso_bwd_arc(const DevGraph &g, const double *__restrict__ f,
                                            const double *__restrict__ h, double *cbar,
                                            const double *__restrict__ Dbar,
                                            double *__restrict__ ubar, int64_t slot, int lane,
                                            double *lds)
{
    constexpr int V = 2;
    int phase = 0;
    const int64_t e = g.aorder[slot];
    const int64_t Kp = g.Kp;
    const int nvec = g.Kp / V;
    const double *fe = f + e * Kp;
    const double *ge = cbar + e * Kp;
    const double *hi = h + (int64_t)g.tails[e] * Kp;
    const double *hj = h + (int64_t)g.heads[e] * Kp;
    const double *Dh = Dbar + (int64_t)g.heads[e] * Kp;
    const double *Dt = Dbar + (int64_t)g.tails[e] * Kp;
    const double u = g.u[e];
    double c[NV][V], gg[NV][V];
    double red[2] = {0.0, 0.0};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            double a[V], b[V], x[V], dh[V], dt[V];
            load_vec_s<true>(fe + q * V, x);
            load_vec(hi + q * V, a);
            load_vec(hj + q * V, b);
            load_vec_s<true>(ge + q * V, gg[v]);
            load_vec(Dh + q * V, dh);
            load_vec(Dt + q * V, dt);
#pragma unroll
            for (int w = 0; w < V; ++w) gg[v][w] = gg[v][w] + dh[w] - dt[w];
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const double cc = 0.5 * ((a[w] + x[w]) - (b[w] - x[w]));
                c[v][w] = cc;
                if (cc > 0.0) {
                    red[0] += cc;
                    red[1] += 1.0;
                }
            }
        } else {
#pragma unroll
            for (int w = 0; w < V; ++w) c[v][w] = gg[v][w] = 0.0;
        }
    }
    group_sum<L, 2>(red, lds, phase);
    double Ssum = red[0], P = red[1];
    double psi = 0.0;
    const bool congested = Ssum > u;
    if (congested) {
        double theta = 0.0;
        for (;;) {
            psi = (Ssum - u) / (1.0 + 0.5 * P);
            const double th = fmax(theta, 0.5 * psi);
            double r2[2] = {0.0, 0.0};
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    const double cc = c[v][w];
                    if (cc > th) {
                        r2[0] += cc;
                        r2[1] += 1.0;
                    }
                }
            group_sum<L, 2>(r2, lds, phase);
            if (r2[1] == P) break;
            Ssum = r2[0];
            P = r2[1];
            theta = th;
        }
    }
    const double half = 0.5 * psi;
    double sa[2] = {0.0, 0.0};  // sum of gbar over A, |A|
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int w = 0; w < V; ++w)
            if (c[v][w] - half > 0.0) {
                sa[0] += gg[v][w];
                sa[1] += 1.0;
            }
    if (congested) group_sum<L, 2>(sa, lds, phase);
    const double share = congested ? sa[0] / (2.0 + sa[1]) : 0.0;
    double *co = cbar + e * Kp;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int q = v * L + lane;
        if (q < nvec) {
            double o[V];
#pragma unroll
            for (int w = 0; w < V; ++w) o[w] = c[v][w] - half > 0.0 ? gg[v][w] - share : 0.0;
            store_vec_s<true>(co + q * V, o);
        }
    }
    if (congested && lane == 0) ubar[e] += share;
}

template <int L, int NV>
__global__ __launch_bounds__(ArcShape<L>::BS) void k_eso_bwd(DevGraph g,
                                                              const double *__restrict__ f,
                                                              const double *__restrict__ h,
                                                              double *cbar,
                                                              const double *__restrict__ Dbar,
                                                              double *__restrict__ ubar)
{
    using S = ArcShape<L>;
    __shared__ double lds[2 * kRedMax * S::NW];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = (L >= S::BS) ? 0 : (int)threadIdx.x / L;
    const int lane = (L >= S::BS) ? (int)threadIdx.x : (int)threadIdx.x & (L - 1);
    const int64_t slot = blk * S::GPB + grp;
    if (L <= 64 && slot >= g.m) return;
    eso_bwd_arc<L, NV>(g, f, h, cbar, Dbar, ubar, slot, lane, lds);
}

// ----------------------------------------------------------------- launch helpers
static inline unsigned grid_for(int64_t work, int64_t cap = 1 << 20)
{
    int64_t b = (work + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

static inline unsigned arc_blocks(int64_t m, int L)
{
    const int BS = L > 64 ? L : 256;
    const int64_t gpb = BS / L;
    return (unsigned)((m + gpb - 1) / gpb);
}


#define PDR_HEIGHT_UNROLL(X) X(1) X(2) X(4) X(8)
#define PDR_TILINGS(X) \
    X(1, 1) X(1, 2) X(1, 4) X(1, 8) \
    X(2, 1) X(2, 2) X(2, 4) X(2, 8) \
    X(4, 1) X(4, 2) X(4, 4) X(4, 8) \
    X(8, 1) X(8, 2) X(8, 4) X(8, 8) \
    X(16, 1) X(16, 2) X(16, 4) X(16, 8) \
    X(32, 1) X(32, 2) X(32, 4) X(32, 8) \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) \
    X(128, 1) X(128, 2) X(128, 4) X(128, 8) X(128, 10) X(128, 12) X(128, 16) X(128, 20) \
    X(256, 1) X(256, 2) X(256, 3) X(256, 4) X(256, 5) X(256, 6) X(256, 8) X(256, 10) \
    X(256, 12) X(256, 16) X(256, 20) \
    X(512, 1) X(512, 2) X(512, 3) X(512, 4) X(512, 5) X(512, 6) X(512, 8) X(512, 10) \
    X(512, 12) \
    X(1024, 1) X(1024, 2) X(1024, 3) X(1024, 4) X(1024, 5) X(1024, 6) X(1024, 8)

}  // namespace pdr
