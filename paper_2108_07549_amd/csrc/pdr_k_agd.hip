// Launcher of the single-context PDR-AGD and PDR-GDM arc kernels.
#include "pdr_device.h"

namespace pdr {

template <typename T, int L, int NV>
static void agd_launch(const DevGraph &g, T *f, const T *h, double *Fsum, double *beta,
                       const AgdParams &prm, const Ctrl *ctrl, T *vel, unsigned nb, hipStream_t st)
{
    constexpr int BS = ArcShape<L>::BS;
    if (vel) {
        if (g.temporal)
            k_gdm<T, L, NV, false><<<nb, BS, 0, st>>>(g, f, vel, h, Fsum, beta, prm, ctrl);
        else
            k_gdm<T, L, NV, true><<<nb, BS, 0, st>>>(g, f, vel, h, Fsum, beta, prm, ctrl);
    } else {
        if (g.temporal)
            k_agd<T, L, NV, false><<<nb, BS, 0, st>>>(g, f, h, Fsum, beta, prm, ctrl);
        else
            k_agd<T, L, NV, true><<<nb, BS, 0, st>>>(g, f, h, Fsum, beta, prm, ctrl);
    }
}

hipError_t launch_agd(const DevGraph &g, bool fp64, Tiling tl, void *f, const void *h,
                      double *Fsum, double *beta, AgdParams prm, const Ctrl *ctrl, void *vel,
                      hipStream_t st)
{
    if (g.m == 0) return hipSuccess;
    if (tl.lanes == kStreamLanes && tl.nv == -kStreamTile) {  // streamed long rows
        if (!g.stream_undo) return hipErrorInvalidValue;
        const unsigned nb = (unsigned)(g.m < kStreamSlots ? g.m : kStreamSlots);
        constexpr int TV = kStreamTile;
        if (fp64 && vel)
            k_agd_stream<double, TV, true><<<nb, kStreamLanes, 0, st>>>(
                g, (double *)f, (double *)vel, (const double *)h, Fsum, beta, prm, ctrl,
                (double *)g.stream_undo);
        else if (fp64)
            k_agd_stream<double, TV, false><<<nb, kStreamLanes, 0, st>>>(
                g, (double *)f, nullptr, (const double *)h, Fsum, beta, prm, ctrl,
                (double *)g.stream_undo);
        else if (vel)
            k_agd_stream<float, TV, true><<<nb, kStreamLanes, 0, st>>>(
                g, (float *)f, (float *)vel, (const float *)h, Fsum, beta, prm, ctrl,
                (float *)g.stream_undo);
        else
            k_agd_stream<float, TV, false><<<nb, kStreamLanes, 0, st>>>(
                g, (float *)f, nullptr, (const float *)h, Fsum, beta, prm, ctrl,
                (float *)g.stream_undo);
        return hipGetLastError();
    }
#define PDR_AGD_CASE(L_, NV_)                                                                  \
    if (tl.lanes == L_ && tl.nv == NV_) {                                                      \
        const unsigned nb = arc_blocks(g.m, L_);                                               \
        if (fp64)                                                                              \
            agd_launch<double, L_, NV_>(g, (double *)f, (const double *)h, Fsum, beta, prm, ctrl, \
                                        (double *)vel, nb, st);                                \
        else                                                                                   \
            agd_launch<float, L_, NV_>(g, (float *)f, (const float *)h, Fsum, beta, prm, ctrl,  \
                                       (float *)vel, nb, st);                                  \
        return hipGetLastError();                                                              \
    }
    PDR_TILINGS(PDR_AGD_CASE)
#undef PDR_AGD_CASE
    return hipErrorInvalidValue;
}


}  // namespace pdr
