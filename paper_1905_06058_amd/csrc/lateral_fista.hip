// FISTA update pass (Alg. 1, Eq. 14, 15) over lateral tiles; the kernel is in lateral.hpp.
#include "lateral.hpp"

namespace isam {

hipError_t lat_fista(const isam_plan_s* p, float2* eh, const float2* gh, float2* z, const float* w,
                     FistaStep fs, float* partials, hipStream_t s) {
    ISAM_LAT_SWITCH(return (launch_fista<N, C>(eh, gh, z, w, p->nk, p->twX[lat_l(p)], fs, partials, s, p->ny,
                                               (unsigned)(p->nx * p->nk))));
}

hipError_t lat_fista_batch(int nx, int sel, int norms, const LatScan* recs, const int2* map, int nblk,
                           const float* beta, hipStream_t s) {
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_C, return (launch_fista_batch<N, C>(norms, recs, map, nblk, beta, s)));
}

}  // namespace isam
