// Host-side context of the library (private): the pdr_ctx record and the
// helpers shared by the single-instance API (pdr_api.cpp) and batches
// (pdr_batch.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "pdr.h"
#include "pdr_internal.h"

namespace pdr_host {
// Text of the calling thread's last failed init (pdr_last_error(NULL)).
extern thread_local std::string g_init_error;
constexpr int kMaxLanes = 1024;
constexpr int kMaxNv = 20;
// Vectors per commodity chunk in the height kernel: small enough that the
// rows read by a window of neighbouring vertices stay in L2.
constexpr int kHeightChunkAuto = 64;
// Blocks of the grid-stride height kernel.
constexpr int kHeightGridAuto = 2048;
// Incident rows each height-kernel thread loads before summing them.
constexpr int kHeightUnrollAuto = 4;
// Vertices per locality cluster of the visiting order.
constexpr int kClusterAuto = 64;
// Blocks of the tiled height kernel: four resident per CU (40 KiB of LDS each).
constexpr int kTileGridAuto = 1024;
// pdr_solve hands FP32 bulk over to the FP64 polish once z is within
// kFloorFactor of the estimated FP32 floor z_noise / rate, the descent rate
// measured over kRateWindows windows (kFloorFactorGdm for GDM, whose FP32
// descent keeps its FP64 pace far below that estimate: measured on a
// 2,500-vertex k-NN instance with 1,000 commodities), or after kStallWindows
// windows without a new lowest z.
constexpr double kFloorFactor = 5.0;
constexpr double kFloorFactorGdm = 0.03;
constexpr int kRateWindows = 4;
constexpr int kStallWindows = 4;
// a window that lowers the lowest z by at most this many z_noise counts as
// no progress
constexpr double kStallNoise = 10.0;
// Flows + heights (+ velocities) of one pass at or below this size are kept
// cache-resident (the MI355X Infinity Cache holds 256 MB).
constexpr double kCacheResidentBytes = 256.0 * 1024.0 * 1024.0;
}  // namespace pdr_host


struct pdr_ctx {
    int32_t n = 0, m = 0, K = 0, Kp = 0;
    int32_t method = PDR_ESO;
    int32_t precision = PDR_FP64;
    pdr_agd_params agd{};
    double beta_min = 0.0;
    double z_feasible_tol = 1e-8;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t req_lanes = 0, req_nv = 0;
    pdr::Tiling tiling{1, 1};
    int32_t graph_sweeps = 32;             // passes per captured graph; 0 = no graphs
    int32_t req_height_chunk = 0;          // 0 = automatic
    int32_t cluster_size = 64;             // vertices per locality cluster; 1 = natural order
    int32_t req_height_grid = 0;           // 0 = automatic
    int32_t req_height_unroll = 0;         // 0 = automatic
    int32_t req_cache_policy = 0;          // 0 = automatic, 1 = ordinary, 2 = non-temporal
    int32_t req_height_kernel = 0;         // 0 = automatic, 1 = vertex-parallel, 2 = tiled
    int32_t ntiles = 0;                    // tiles of the tiled height kernel (0: not used)
    hipStream_t cap_stream = nullptr;      // private stream used only for capture
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // one per precision
    bool poisoned = false;
    std::string err;

    pdr::DevGraph g{};
    // instance arrays (device)
    int32_t *d_row_ptr = nullptr, *d_tails = nullptr, *d_heads = nullptr, *d_in_ptr = nullptr,
            *d_in_idx = nullptr, *d_deg = nullptr, *d_inj_ptr = nullptr, *d_inj_k = nullptr,
            *d_s = nullptr, *d_t = nullptr, *d_vorder = nullptr, *d_aorder = nullptr,
            *d_vinfo = nullptr, *d_vinc = nullptr, *d_tinfo = nullptr, *d_tarc = nullptr;
    uint16_t *d_tslot = nullptr;
    double *d_inj_val = nullptr, *d_u = nullptr, *d_d = nullptr;
    // run state (device)
    double *f64 = nullptr, *h64 = nullptr, *v64 = nullptr;
    double *d_undo = nullptr;              // undo rows of the streamed AGD / GDM kernels
    float *f32 = nullptr, *h32 = nullptr, *v32 = nullptr;
    double *Fsum = nullptr, *beta = nullptr, *zpart = nullptr, *maxpart = nullptr,
           *arcpart = nullptr, *resout = nullptr, *zlog = nullptr;
    int64_t nzpart = 0;
    int64_t zlog_cap = pdr::kZLogCap;      // entries of the z log ring (power of two)
    bool batch_member = false;             // owned by a pdr_batch
    pdr::Ctrl *ctrl = nullptr;
    // pdr_solve's hand-over tracking, carried from one call to the next:
    // lowest z and passes of the recent FP32 windows, consecutive windows
    // without a new lowest z, and the lowest z before the current window.
    // Reset when the state or the precision is replaced.
    struct SolveTrack {
        std::vector<std::pair<double, int64_t>> recent;
        int stalled = 0;
        double best_before = HUGE_VAL;
    } solve_track;
    // pinned host mirrors
    pdr::Ctrl *h_ctrl = nullptr;
    double *h_res = nullptr;
    std::vector<void *> allocs;
};


namespace pdr_host {
int pow2ceil(int64_t x);
void *cur_f(pdr_ctx *c);  // flows, heights, velocities in the storage precision
void *cur_h(pdr_ctx *c);
void *cur_v(pdr_ctx *c);
pdr::AgdParams agd_params(const pdr_ctx *c);
// Switch a context's storage precision (pdr_set_precision without the check
// that refuses batch members).
pdr_status set_precision_impl(pdr_ctx *c, int32_t precision);
// Choose the sweep kernels' cache hints for the current storage precision
// (batch members always stream).
void set_cache_policy(pdr_ctx *c);
// pdr_set_state's argument checks (the text goes to c->err).
pdr_status check_state_args(pdr_ctx *c, const double *f, const double *beta, const double *v,
                            int64_t t, double z_prev);
// pdr_set_state after its checks, staging the host rows through `staging`
// (device memory of staging_doubles doubles, at least one row of K) in chunks
// of whole rows; allocates nothing. Synchronizes.
pdr_status set_state_impl(pdr_ctx *c, const double *f, const double *beta, const double *v,
                          int64_t t, double z_prev, double *staging, int64_t staging_doubles);
// The device address of the file-scope staging array of pdr_set_state_noalloc
// on `device` (resolved once per device; the device must be current).
hipError_t noalloc_scratch(int device, double **out, int64_t *doubles);

// Exception barrier of the C ABI: every exported entry point runs its body
// through abi_guard, so no C++ exception (in practice std::bad_alloc from a
// host container) leaves the library. A failed host allocation returns
// PDR_ERR_OOM, any other exception PDR_ERR_INVALID; the text goes to *err (to
// the calling thread's init error when err is NULL). A call that may have
// changed the object's state part way passes the object's poisoned flag,
// which is then set: later calls answer PDR_ERR_DEVICE until it is destroyed.
template <typename Body>
pdr_status abi_guard(std::string *err, bool *poisoned, Body &&body) noexcept
{
    pdr_status st = PDR_ERR_INVALID;
    const char *what = "unexpected C++ exception";
    try {
        return body();
    } catch (const std::bad_alloc &) {
        st = PDR_ERR_OOM;
        what = "host memory allocation failed";
    } catch (const std::length_error &) {
        st = PDR_ERR_OOM;
        what = "host allocation larger than the address space";
    } catch (...) {
    }
    if (poisoned) *poisoned = true;
    try {
        std::string &dst = err ? *err : g_init_error;
        dst = what;
        if (poisoned) dst += " (the object is poisoned; destroy it)";
    } catch (...) {
    }
    return st;
}
}  // namespace pdr_host
