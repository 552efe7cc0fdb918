// FISTA update pass (Alg. 1, Eq. 14, 15) over lateral tiles; the kernel is in lateral.hpp.
#include "lateral.hpp"

namespace isam {

hipError_t lat_fista(const isam_plan_s* p, float2* eh, const float2* gh, float2* z, const float* w,
                     FistaStep fs, float* partials, hipStream_t s) {
    ISAM_LAT_SWITCH(return (launch_fista<N, C>(eh, gh, z, w, p->nk, p->twX[lat_l(p)], fs, partials, s)));
}

}  // namespace isam
