// Boxes of the FP32 barycenters of kTileJ-face tiles (FaceData::tbox) and the tests the
// all-pairs kernels make with them.
#pragma once
#include "tp_internal.h"

namespace tp {

// Box of the i-range [ibase, ibase + ispan) from the tile boxes.
__device__ __forceinline__ void irange_box(const float4* tbox, int64_t ibase, int ispan, float4& lo, float4& hi)
{
    lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
    hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
    for (int64_t t = ibase / kTileJ; t < (ibase + ispan) / kTileJ; ++t) {
        const float4 a = tbox[2 * t], b = tbox[2 * t + 1];
        lo = make_float4(fminf(lo.x, a.x), fminf(lo.y, a.y), fminf(lo.z, a.z), 0.f);
        hi = make_float4(fmaxf(hi.x, b.x), fmaxf(hi.y, b.y), fmaxf(hi.z, b.z), 0.f);
    }
}

// Far tiles drop the low parts of the barycenters.  Without them the difference of two
// barycenters carries an absolute error of at most 2^-24 (|X_S| + |X_T|) per coordinate
// (the rounding of X to FP32) instead of 2^-24 |X_S - X_T| with them.  When every pair of
// the i-range box and the j-tile box is at least kFarRatio x the largest coordinate
// magnitude of the two boxes apart, that error is at most 2 / kFarRatio = 8 times the
// rounding of the hi/lo difference: a relative error of at most 8 x 2^-24 in d, hence of a
// few 1e-6 at most in a pair term r2^-e q^m with e, m <= 6 (and most far terms are small:
// they fall off as |d|^-7 for the energy, |d|^-(2 sigma + 2) and |d|^-2s for the operators).
constexpr float kFarRatio = 0.25f;

__device__ __forceinline__ bool tile_is_far(const float4& ilo, const float4& ihi, const float4* tbox, int jt)
{
    const float4 a = tbox[2 * jt], b = tbox[2 * jt + 1];
    const float gx = fmaxf(fmaxf(a.x - ihi.x, ilo.x - b.x), 0.f);
    const float gy = fmaxf(fmaxf(a.y - ihi.y, ilo.y - b.y), 0.f);
    const float gz = fmaxf(fmaxf(a.z - ihi.z, ilo.z - b.z), 0.f);
    const float m = fmaxf(fmaxf(fmaxf(fabsf(a.x), fabsf(b.x)), fmaxf(fabsf(a.y), fabsf(b.y))),
                          fmaxf(fmaxf(fabsf(a.z), fabsf(b.z)),
                                fmaxf(fmaxf(fmaxf(fabsf(ilo.x), fabsf(ihi.x)), fmaxf(fabsf(ilo.y), fabsf(ihi.y))),
                                      fmaxf(fabsf(ilo.z), fabsf(ihi.z)))));
    const float g2 = gx * gx + gy * gy + gz * gz;
    // An empty box (a tile of padding faces) gives g2 = m = inf and counts as far: its
    // zero-area faces add nothing on either path.
    return g2 >= (kFarRatio * kFarRatio) * (m * m);
}

}  // namespace tp
