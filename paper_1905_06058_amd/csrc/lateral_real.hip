// Lateral real transforms: C2R (real projection of Eq. 5) and R2C (lateral spectrum of real
// spectra); the kernels are in lateral.hpp.
#include "lateral.hpp"

namespace isam {

int lat_l_real(const isam_plan_s* p) {
    ISAM_LAT_SWITCH_R(return (LatCfg<N, C>::L));
}

// Per A-scan row (for a volume: per slab, half spectra [nh][nk] blocked per slab).
hipError_t lat_c2r(const isam_plan_s* p, const float2* zh, float* sout, hipStream_t s) {
    const unsigned sh = (unsigned)(p->nh * p->nk), sf = (unsigned)(p->nx * p->nk);
    ISAM_LAT_SWITCH_R(return (launch_c2r<N, C>(zh, sout, p->nk, p->twX[lat_l_real(p)], s, p->ny, sh, sf)));
}

hipError_t lat_r2c(const isam_plan_s* p, const float* r, float2* rh, hipStream_t s) {
    const unsigned sh = (unsigned)(p->nh * p->nk), sf = (unsigned)(p->nx * p->nk);
    ISAM_LAT_SWITCH_R(return (launch_r2c<N, C>(r, rh, p->nk, p->twX[lat_l_real(p)], s, p->ny, sf, sh)));
}

hipError_t lat_c2r_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, hipStream_t s) {
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_CR, return (launch_c2r_batch<N, C>(recs, map, nblk, s)));
}

hipError_t lat_r2c_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, hipStream_t s) {
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_CR, return (launch_r2c_batch<N, C>(recs, map, nblk, s)));
}

}  // namespace isam
