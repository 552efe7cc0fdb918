// Lateral complex transforms (the lateral DFT of Eq. 2, 16, 17) and the lateral-length
// dispatch shared by all lateral passes; the kernels are in lateral.hpp.
#include "lateral.hpp"

namespace isam {

bool lat_supported(int nx) {
    switch (nx) {
        case 1: case 2: case 4: case 8: case 16: case 32: case 64: case 128:
        case 192: case 256: case 320: case 384: case 448: case 512: case 640: case 768:
        case 896: case 1024: case 1280: case 1536: case 1792: case 2048:
            return true;
        default:
            return false;
    }
}

// Radix cap (log2) of the lateral FFT in use: selects the matching staged twiddle table.
int lat_l(const isam_plan_s* p) {
    ISAM_LAT_SWITCH(return (LatCfg<N, C>::L));
}
// x transform of every A-scan row (for a volume: of each of the ny slabs [nx][nk]).
hipError_t lat_c2c(const isam_plan_s* p, const float2* in, float2* out, int sign, hipStream_t s) {
    const unsigned slab = (unsigned)(p->nx * p->nk);
    ISAM_LAT_SWITCH(return (launch_c2c<N, C>(in, out, p->nk, p->twX[lat_l(p)], sign, s, p->ny, slab, slab)));
}

// y transform of a volume: length ny over ncols columns (row-major [ny][ncols] <-> blocked).
hipError_t lat_c2c_y(const isam_plan_s* p, const float2* in, float2* out, int ncols, int sign, hipStream_t s) {
    // wide tiles (16 lanes, 128 bytes per row) up to 512 rows: the rows are far apart in memory
    ISAM_LAT_DISPATCH(p->ny, p->lat_cy, (N <= 256 ? 32 : N <= 512 ? 16 : ISAM_LAT_DEF_C),
                      return (launch_c2c<N, C>(in, out, ncols, p->twY[LatCfg<N, C>::L], sign, s, 1, 0u, 0u)));
}

int lat_blocks(const isam_plan_s* p, int kind) {
    if (kind == 0) {
        ISAM_LAT_SWITCH((void)N; return p->ny * (p->nk / C));
    }
    ISAM_LAT_SWITCH_R((void)N; return p->ny * (p->nk / (2 * C)));
}

int lat_tile(int nx, int sel, int real) {
    if (real) {
        ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_CR, (void)N; return C);
    }
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_C, (void)N; return C);
}

int lat_radix_cap(int nx, int sel, int real) {
    if (real) {
        ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_CR, return (LatCfg<N, C>::L));
    }
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_C, return (LatCfg<N, C>::L));
}

hipError_t lat_c2c_batch(int nx, int sel, const LatScan* recs, const int2* map, int nblk, int sign, hipStream_t s) {
    ISAM_LAT_DISPATCH(nx, sel, ISAM_LAT_DEF_C, return (launch_c2c_batch<N, C>(recs, map, nblk, sign, s)));
}

}  // namespace isam
