// Internal interface between the host library (pdr_api.cpp) and the HIP
// kernels (pdr_device.h and the pdr_k_*.hip translation units). Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdr {

// Device-resident run control and scalar state, read and written by the
// kernels so that a sweep never needs a host round trip.
struct Ctrl {
    int32_t stopped;     // the stop test fired in the current pdr_sweep call
    int32_t numeric;     // the objective was non-finite
    int64_t t;           // iteration counter: arc updates applied so far
    int64_t t_pass;      // iteration index used by the current pass's arc update
    int64_t evals;       // number of objective evaluations logged
    double z_prev;       // previous objective (stop test of Algorithm 1)
    double eps_obj;      // stop if |z - z_prev| < eps_obj (when > 0)
    double z_target;     // stop if z <= z_target (when > 0)
    double z, z_psi, z_h;  // last evaluated objective and its two parts
    double z_noise;        // FP32 storage: objective left by rounding the flows alone
};

constexpr int64_t kZLogCap = int64_t(1) << 20;
// The height kernel is grid-stride with at most this many blocks (8 per CU),
// which also bounds the number of objective partials.
constexpr int64_t kHeightBlocksMax = 8192;

// Graph and instance arrays in device memory.
struct DevGraph {
    int32_t n, m, K, Kp;
    int32_t height_cv;       // vectors per commodity chunk in the height kernel
    int32_t height_grid;     // blocks of the height kernel (<= kHeightBlocksMax)
    int32_t height_unroll;   // incident rows loaded together per thread (1, 2 or 4)
    const int32_t *row_ptr;  // n+1: out-arcs of i are [row_ptr[i], row_ptr[i+1])
    const int32_t *tails;    // m
    const int32_t *heads;    // m
    const int32_t *in_ptr;   // n+1: in-arcs of i are in_idx[in_ptr[i] .. in_ptr[i+1])
    const int32_t *in_idx;   // m, ascending arc ids per head
    const int32_t *deg;      // n: in-degree + out-degree
    const int32_t *inj_ptr;  // n+1: injections of vertex i
    const int32_t *inj_k;    // 2K: commodity of each injection, ascending per vertex
    const double *inj_val;   // 2K: +d_k at s_k, -d_k at t_k
    const double *u;         // m capacities
    const int32_t *s, *t;    // K
    const double *d;         // K
    const int32_t *vorder;   // n: order in which the height kernel visits vertices
    const int32_t *aorder;   // m: order in which the arc kernels visit arcs
    // Incidence lists in visiting order: position p of vorder has
    // vinfo[8p .. 8p+3] = (vertex i, first, number of in-arcs, end) and its
    // arcs are vinc[first .. end): in-arcs in ascending id, then out-arcs in
    // ascending id (end - first = delta_i); vinfo[8p+4 .. 8p+7] =
    // (inj_ptr[i], inj_ptr[i+1], smallest and largest commodity injected at
    // i; K and -1 if none).
    const int32_t *vinfo;    // 8n, 16-byte aligned
    const int32_t *vinc;     // 2m
    // 1: a pass's flows, heights and velocities fit in the Infinity Cache, so
    // the sweep kernels use ordinary loads and stores and the data stays
    // resident between passes; 0: they stream with non-temporal hints.
    int32_t temporal;
    // Tiles of the tiled height kernel (ntiles 0: the vertex-parallel kernel
    // runs instead). Tile t covers visiting positions [tinfo[4t], tinfo[4t+1])
    // and the arcs tarc[tinfo[4t+2] .. tinfo[4t+3]) incident to them (each
    // once); tslot[p] is the index of arc vinc[p] in its vertex's tile list.
    // Undo rows of the streamed AGD / GDM kernels: (GDM ? 2 : 1) rows of Kp
    // FP64-sized elements for each of their kStreamSlots blocks (null unless
    // the context's rows are streamed and the method is AGD or GDM).
    void *stream_undo;
    int32_t ntiles;
    int32_t tile_grid;       // blocks of the tiled height kernel
    const int32_t *tinfo;    // 4 * ntiles, 16-byte aligned
    const int32_t *tarc;
    const uint16_t *tslot;   // 2m, parallel to vinc
};

// Tiled height kernel: at most kTileVerts vertices and kTileArcs incident arcs
// per tile; a block stages kTileVecs 16-byte vectors of each arc in LDS.
constexpr int kTileVerts = 64;
constexpr int kTileArcs = 304;
constexpr int kTileVecs = 8;

struct AgdParams {
    double beta_min, beta_max, alpha_inc, alpha_dec;
    int32_t inc_period;
    double gamma;  // momentum (GDM)
};

// Arc-kernel tiling: `lanes` lanes cooperate on one arc, each holding up to
// `nv` 16-byte vectors of the arc's commodity row in registers. A negative nv
// names the streamed kernels for rows longer than any resident tiling: the
// lanes pass over the row in tiles of lanes x (-nv) vectors (Tiling{1024, -4},
// streamed_tiling()).
struct Tiling {
    int lanes;
    int nv;
};
// The one streamed tiling.
Tiling streamed_tiling();
// Blocks of the streamed AGD / GDM kernels, each with its own undo rows.
constexpr int kStreamSlots = 256;

// One instance of a batch as the batched kernels see it (device-resident
// array, one entry per instance). All instances of a batch share one storage
// precision; f, h and v point into that instance's own buffers.
struct InstView {
    DevGraph g;
    void *f, *h, *v;        // flows, heights, GDM velocities (v null unless GDM)
    double *Fsum, *beta;
    AgdParams prm;          // AGD/GDM parameters (beta_min depends on K)
    Ctrl *ctrl;
    double *zpart;          // 3 * nzpart objective partials
    double *zlog;           // z log ring of zmask + 1 entries
    int64_t zmask;
    int32_t nzpart;         // height blocks of this instance in a batched pass
};

bool tiling_supported(int lanes, int nv);
// Longest row, in 16-byte vectors, that some supported tiling covers.
int max_tiling_vectors();
int64_t height_blocks(const DevGraph &g, int elem_bytes);

// Launchers; each returns the launch status.
hipError_t launch_begin(Ctrl *ctrl, double eps_obj, double z_target, hipStream_t st);
// Heights of the current flows, then the objective and stop test (two kernels).
hipError_t launch_height(const DevGraph &g, bool fp64, const void *f, void *h, double *zpart,
                         const double *Fsum, Ctrl *ctrl, double *zlog, int64_t zmask,
                         hipStream_t st);
hipError_t launch_height_resid(const DevGraph &g, bool fp64, const void *f, double *h64,
                               double *zpart, double *maxpart, hipStream_t st);
// ESO arc update (Expression 14); cap: the capacity-enforcing step instead.
hipError_t launch_eso(const DevGraph &g, bool fp64, Tiling tl, void *f, const void *h,
                      double *Fsum, const Ctrl *ctrl, bool cap, hipStream_t st);
// One FP64 ESO pass reading fin and writing fout (distinct buffers), no stop
// test (the adjoint's segment recomputation).
hipError_t launch_eso_oop(const DevGraph &g, Tiling tl, const double *fin, double *fout,
                          const double *h, double *Fsum, hipStream_t st);
// AGD arc update (Algorithm 3); with a velocity buffer vel, the GDM update
// (Algorithm 4).
hipError_t launch_agd(const DevGraph &g, bool fp64, Tiling tl, void *f, const void *h,
                      double *Fsum, double *beta, AgdParams prm, const Ctrl *ctrl, void *vel,
                      hipStream_t st);
hipError_t launch_rowsum(const DevGraph &g, bool fp64, Tiling tl, const void *f, double *Fsum,
                         hipStream_t st);
// Residual report: per-arc partials then one final reduction into out[8].
hipError_t launch_resid(const DevGraph &g, bool fp64, const void *f, const double *h64,
                        const double *Fsum, const double *zpart, int64_t nzpart,
                        const double *maxpart, double *arcpart, double *out,
                        hipStream_t st);
hipError_t launch_copy(const void *src, void *dst, int64_t count16, hipStream_t st);
hipError_t launch_convert(const void *src, bool src_fp64, void *dst, bool dst_fp64,
                          int64_t count, hipStream_t st);
// Unpadded copy of flows: dst[e*K + k] = f[e*Kp + k].
hipError_t launch_unpad(const DevGraph &g, const void *f, bool f_fp64, void *dst, bool dst_fp64,
                        hipStream_t st);
hipError_t launch_pad(const DevGraph &g, const double *src, void *f, bool f_fp64,
                      hipStream_t st);
// Rows [row0, row0 + rows) of f from src holding just those rows, unpadded.
hipError_t launch_pad_rows(const DevGraph &g, const double *src, void *f, bool f_fp64,
                           int64_t row0, int64_t rows, hipStream_t st);

// Reverse mode through FP64 PDR-ESO passes. Seed at the final flows (Fsum and
// h of those flows): cbar = dz/df (to be read with Dbar = 0), ubar = dz/du and
// dbar = dz/dd (the direct terms).
hipError_t launch_adj_seed(const DevGraph &g, const double *Fsum, const double *h, double *cbar,
                           double *ubar, double *dbar, hipStream_t st);
// One pass in reverse: f and h are the pass's input flows and heights; on
// entry dz/df of the pass's output is cbar + Dbar_head - Dbar_tail; on return
// cbar and Dbar hold the pass's own, and ubar and dbar have accumulated. tl is
// the tiling the forward arc kernel used.
// The vertex half of launch_adj_pass (Dbar from cbar, then dbar).
hipError_t launch_adj_vertex(const DevGraph &g, const double *cbar, double *Dbar, double *dbar,
                             hipStream_t st);
hipError_t launch_adj_pass(const DevGraph &g, Tiling tl, const double *f, const double *h,
                           double *cbar, double *Dbar, double *ubar, double *dbar, hipStream_t st);

// Batched passes over B instances (views: device array of B InstView).
// hmap / amap: per logical block, (instance, block within that instance).
hipError_t launch_bbegin(const InstView *views, int B, double eps_obj, double z_target,
                         hipStream_t st);
hipError_t launch_bheight(const InstView *views, int B, const int2 *hmap, int64_t nblocks,
                          bool fp64, int unroll, hipStream_t st);
// method: 0 ESO, 1 AGD, 2 GDM, 3 capacity-enforcing; blocks of `amap` hold
// ArcShape(tl.lanes) groups.
hipError_t launch_barc(int method, const InstView *views, const int2 *amap, int64_t nblocks,
                       bool fp64, Tiling tl, hipStream_t st);
// Number of instances whose stop test has fired (written to device *out).
hipError_t launch_bcount_stopped(const InstView *views, int B, int32_t *out, hipStream_t st);
// Arcs handled by one block of an arc kernel with `lanes` lanes per arc.
int arcs_per_block(int lanes);

}  // namespace pdr
