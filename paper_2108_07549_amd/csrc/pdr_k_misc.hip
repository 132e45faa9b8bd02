// Launchers of the row-sum, out-of-place ESO and reverse ESO arc kernels.
#include "pdr_device.h"

namespace pdr {

hipError_t launch_eso_oop(const DevGraph &g, Tiling tl, const double *fin, double *fout,
                          const double *h, double *Fsum, hipStream_t st)
{
    if (g.m == 0) return hipSuccess;
#define PDR_OOP_CASE(L_, NV_)                                                                   \
    if (tl.lanes == L_ && tl.nv == NV_) {                                                       \
        k_eso_oop<L_, NV_><<<arc_blocks(g.m, L_), ArcShape<L_>::BS, 0, st>>>(g, fin, fout, h,   \
                                                                              Fsum);            \
        return hipGetLastError();                                                               \
    }
    PDR_TILINGS(PDR_OOP_CASE)
#undef PDR_OOP_CASE
    return hipErrorInvalidValue;
}

// Row sums use the tiling of the arc kernels, chosen by the caller.
hipError_t launch_rowsum(const DevGraph &g, bool fp64, Tiling tl, const void *f, double *Fsum,
                         hipStream_t st)
{
    if (g.m == 0) return hipSuccess;
    if (tl.lanes == kStreamLanes && tl.nv == -kStreamTile) {  // streamed long rows
        if (fp64)
            k_rowsum_stream<double, kStreamTile><<<(unsigned)g.m, kStreamLanes, 0, st>>>(g, (const double *)f, Fsum);
        else
            k_rowsum_stream<float, kStreamTile><<<(unsigned)g.m, kStreamLanes, 0, st>>>(g, (const float *)f, Fsum);
        return hipGetLastError();
    }
#define PDR_ROW_CASE(L_, NV_)                                                                    \
    if (tl.lanes == L_ && tl.nv == NV_) {                                                        \
        const unsigned nb = arc_blocks(g.m, L_);                                                 \
        constexpr int BS = L_ > 64 ? L_ : 256;                                                   \
        if (fp64)                                                                                \
            k_rowsum<double, L_, NV_><<<nb, BS, 0, st>>>(g, (const double *)f, Fsum);            \
        else                                                                                     \
            k_rowsum<float, L_, NV_><<<nb, BS, 0, st>>>(g, (const float *)f, Fsum);              \
        return hipGetLastError();                                                                \
    }
    PDR_TILINGS(PDR_ROW_CASE)
#undef PDR_ROW_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_adj_pass(const DevGraph &g, Tiling tl, const double *f, const double *h,
                           double *cbar, double *Dbar, double *ubar, double *dbar, hipStream_t st)
{
    if (g.m > 0) {
        bool launched = false;
#define PDR_AB(L_, NV_)                                                                        \
    if (!launched && tl.lanes == L_ && tl.nv == NV_) {                                         \
        constexpr int BS = L_ > 64 ? L_ : 256;                                                 \
        k_eso_bwd<L_, NV_><<<arc_blocks(g.m, L_), BS, 0, st>>>(g, f, h, cbar, Dbar, ubar);     \
        launched = true;                                                                       \
    }
        PDR_TILINGS(PDR_AB)
#undef PDR_AB
        if (!launched) return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_adj_vertex(g, cbar, Dbar, dbar, st);
}


}  // namespace pdr
