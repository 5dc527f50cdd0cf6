// Tile enumeration of the trailing update C := C - X^T Y (host and device).
//
// C is cut into 128 x 128 tiles, tm x tn of them.  With `upper` only tiles
// that touch the upper triangle (I <= J) exist.  Tiles are numbered band by
// band: a band is G consecutive tile rows; inside a band the order is
// column-major (all band rows of tile column J, then J + 1, ...).  Tiles that
// run at the same time therefore share a few column slabs of X and Y, which
// keeps those slabs resident in one XCD's L2.  Workgroups are dealt to the
// eight XCDs round-robin; xcd_remap hands each XCD a contiguous run of this
// order.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define FLAME_HD
#else
#define FLAME_HD __host__ __device__
#endif

namespace flame {

constexpr int kTile = 128;
constexpr int kBand = 8;
constexpr int kXcds = 8;

FLAME_HD inline int64_t band_tiles(int beta, int tm, int tn, bool upper) {
    const int i0 = beta * kBand;
    const int hb = (tm - i0 < kBand) ? (tm - i0) : kBand;
    if (hb <= 0) return 0;
    if (!upper) return (int64_t)hb * tn;
    const int L = tn - i0;  // tile columns J >= i0
    if (L <= 0) return 0;
    if (L <= hb - 1) return (int64_t)L * (L + 1) / 2;
    return (int64_t)hb * (hb - 1) / 2 + (int64_t)(L - (hb - 1)) * hb;
}

FLAME_HD inline int64_t tile_count(int tm, int tn, bool upper) {
    int64_t c = 0;
    const int nbands = (tm + kBand - 1) / kBand;
    for (int b = 0; b < nbands; ++b) c += band_tiles(b, tm, tn, upper);
    return c;
}

// t in [0, tile_count) -> (I, J).
FLAME_HD inline void tile_of(int64_t t, int tm, int tn, bool upper, int &I, int &J) {
    const int nbands = (tm + kBand - 1) / kBand;
    for (int beta = 0; beta < nbands; ++beta) {
        const int64_t c = band_tiles(beta, tm, tn, upper);
        if (t < c) {
            const int i0 = beta * kBand;
            const int hb = (tm - i0 < kBand) ? (tm - i0) : kBand;
            if (!upper) {
                J = (int)(t / hb);
                I = i0 + (int)(t % hb);
                return;
            }
            const int64_t tri = (int64_t)hb * (hb - 1) / 2;
            if (t < tri) {
                // triangle part: band column jj has jj + 1 tiles
                int jj = 0;
                while ((int64_t)(jj + 1) * (jj + 2) / 2 <= t) ++jj;
                J = i0 + jj;
                I = i0 + (int)(t - (int64_t)jj * (jj + 1) / 2);
            } else {
                const int64_t u = t - tri;
                J = i0 + hb - 1 + (int)(u / hb);
                I = i0 + (int)(u % hb);
            }
            return;
        }
        t -= c;
    }
    I = J = -1;
}

// Workgroup id -> position in the band order, so that XCD x (which receives
// ids x, x + 8, x + 16, ...) works on one contiguous run of tiles.
FLAME_HD inline int64_t xcd_remap(int64_t w, int64_t nt) {
    const int64_t q = nt / kXcds, r = nt % kXcds;
    const int64_t x = w % kXcds, i = w / kXcds;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace flame
