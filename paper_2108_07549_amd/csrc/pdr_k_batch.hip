// Launcher of the batched arc kernels (every method and precision).
#include "pdr_device.h"

namespace pdr {

hipError_t launch_barc(int method, const InstView *views, const int2 *amap, int64_t nblocks,
                       bool fp64, Tiling tl, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned nb = (unsigned)nblocks;
#define PDR_BA(L_, NV_)                                                                        \
    if (tl.lanes == L_ && tl.nv == NV_) {                                                      \
        constexpr int BS = L_ > 64 ? L_ : 256;                                                 \
        if (method == 0 && fp64)                                                               \
            kb_eso<double, L_, NV_, false><<<nb, BS, 0, st>>>(views, amap);                    \
        else if (method == 0)                                                                  \
            kb_eso<float, L_, NV_, false><<<nb, BS, 0, st>>>(views, amap);                     \
        else if (method == 3 && fp64)                                                          \
            kb_eso<double, L_, NV_, true><<<nb, BS, 0, st>>>(views, amap);                     \
        else if (method == 3)                                                                  \
            kb_eso<float, L_, NV_, true><<<nb, BS, 0, st>>>(views, amap);                      \
        else if (method == 1 && fp64)                                                          \
            kb_agd<double, L_, NV_><<<nb, BS, 0, st>>>(views, amap);                           \
        else if (method == 1)                                                                  \
            kb_agd<float, L_, NV_><<<nb, BS, 0, st>>>(views, amap);                            \
        else if (fp64)                                                                         \
            kb_gdm<double, L_, NV_><<<nb, BS, 0, st>>>(views, amap);                           \
        else                                                                                   \
            kb_gdm<float, L_, NV_><<<nb, BS, 0, st>>>(views, amap);                            \
        return hipGetLastError();                                                              \
    }
    PDR_TILINGS(PDR_BA)
#undef PDR_BA
    return hipErrorInvalidValue;
}


}  // namespace pdr
