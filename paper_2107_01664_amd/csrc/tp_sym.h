// Pieces shared by the symmetric all-pairs kernels, which evaluate each unordered pair of
// faces once for both rows: blocks of faces, the pairs of blocks of a band of rows, and
// the rotation of values along a wave.
#pragma once
#include "tp_internal.h"

namespace tp {

constexpr int kSymNI = 4;                 // faces S per lane
constexpr int kSymFaces = 64 * kSymNI;    // faces per block: one wave's faces S

// Value of the lane one below (lane 0 takes lane 63's): a rotation of the whole wave through
// the LDS crossbar (ds_bpermute).  The pair loops are bound by vector-ALU issue, and a DPP
// move would take an issue slot per value (one that another wave's instruction cannot
// share, measured); ds_bpermute takes none, only LDS bandwidth, which these loops leave idle.
struct WaveRot {
    int addr;   // byte address of the source lane
    __device__ __forceinline__ explicit WaveRot(int lane) : addr(((lane + 63) & 63) << 2) {}
    __device__ __forceinline__ int operator()(int v) const { return __builtin_amdgcn_ds_bpermute(addr, v); }
    __device__ __forceinline__ float operator()(float v) const
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
    }
};

// Pairs of blocks (a, b), b >= a, with a in the band [a0, a1): the off-diagonal ones
// (a < b) first, row by row, then the diagonal ones, which do one side only and so make a
// lighter last round.
__host__ __device__ __forceinline__ int64_t sym_band_offdiag(int nB, int a0, int a1)
{
    // sum over a in [a0, a1) of nB - 1 - a
    return (int64_t)(a1 - a0) * (nB - 1) - ((int64_t)a1 * (a1 - 1) - (int64_t)a0 * (a0 - 1)) / 2;
}

__device__ __forceinline__ bool sym_unit_blocks(int64_t unit, int nB, int a0, int a1, int& a, int& b)
{
    const int64_t noff = sym_band_offdiag(nB, a0, a1);
    if (unit >= noff) {
        a = b = a0 + (int)(unit - noff);
        return a < a1;
    }
    a = a0;
    int64_t off = 0;
    while (off + (nB - 1 - a) <= unit) {
        off += nB - 1 - a;
        ++a;
    }
    b = a + 1 + (int)(unit - off);
    return true;
}

}  // namespace tp
