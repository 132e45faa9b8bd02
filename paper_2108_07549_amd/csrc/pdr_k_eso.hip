// Launcher of the single-context PDR-ESO and capacity-enforcing arc kernels.
#include "pdr_device.h"

namespace pdr {

// The single-context sweep kernels come in two cache-hint variants; the
// graph's `temporal` flag picks one (DevGraph::temporal).
template <typename T, int L, int NV>
static void eso_launch(const DevGraph &g, T *f, const T *h, double *Fsum, const Ctrl *ctrl,
                       bool cap, unsigned nb, hipStream_t st)
{
    constexpr int BS = ArcShape<L>::BS;
    if (g.temporal) {
        if (cap) k_eso<T, L, NV, true, false><<<nb, BS, 0, st>>>(g, f, h, Fsum, ctrl);
        else k_eso<T, L, NV, false, false><<<nb, BS, 0, st>>>(g, f, h, Fsum, ctrl);
    } else {
        if (cap) k_eso<T, L, NV, true, true><<<nb, BS, 0, st>>>(g, f, h, Fsum, ctrl);
        else k_eso<T, L, NV, false, true><<<nb, BS, 0, st>>>(g, f, h, Fsum, ctrl);
    }
}

hipError_t launch_eso(const DevGraph &g, bool fp64, Tiling tl, void *f, const void *h,
                      double *Fsum, const Ctrl *ctrl, bool cap, hipStream_t st)
{
    if (g.m == 0) return hipSuccess;
    if (tl.lanes == kStreamLanes && tl.nv == -kStreamTile) {  // streamed long rows
        const unsigned nb = (unsigned)g.m;
        constexpr int TV = kStreamTile;
        if (fp64 && cap)
            k_eso_stream<double, TV, true><<<nb, kStreamLanes, 0, st>>>(g, (double *)f, (const double *)h, Fsum, ctrl);
        else if (fp64)
            k_eso_stream<double, TV, false><<<nb, kStreamLanes, 0, st>>>(g, (double *)f, (const double *)h, Fsum, ctrl);
        else if (cap)
            k_eso_stream<float, TV, true><<<nb, kStreamLanes, 0, st>>>(g, (float *)f, (const float *)h, Fsum, ctrl);
        else
            k_eso_stream<float, TV, false><<<nb, kStreamLanes, 0, st>>>(g, (float *)f, (const float *)h, Fsum, ctrl);
        return hipGetLastError();
    }
#define PDR_ESO_CASE(L_, NV_)                                                                    \
    if (tl.lanes == L_ && tl.nv == NV_) {                                                        \
        const unsigned nb = arc_blocks(g.m, L_);                                                 \
        if (fp64)                                                                                \
            eso_launch<double, L_, NV_>(g, (double *)f, (const double *)h, Fsum, ctrl, cap, nb,   \
                                        st);                                                     \
        else                                                                                     \
            eso_launch<float, L_, NV_>(g, (float *)f, (const float *)h, Fsum, ctrl, cap, nb, st); \
        return hipGetLastError();                                                                \
    }
    PDR_TILINGS(PDR_ESO_CASE)
#undef PDR_ESO_CASE
    return hipErrorInvalidValue;
}


}  // namespace pdr
