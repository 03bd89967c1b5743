// Walk of the heap-ordered Barnes-Hut tree by a whole wave (64 lanes) at once.
//
// Each lane has its own interaction list (its own admissibility tests), but the lanes of a
// wave hold neighbouring faces in Morton order, so their lists overlap.  The wave visits a
// node when at least one of its lanes needs it, in the order of a single depth-first walk
// (left child first), so every lane meets the terms of its own list in the order it would
// walking alone, and all lanes read the same node at the same time.  A lane that takes a
// node -- far(node) when the node is admissible for it, near(node) for a leaf that is not --
// skips the node's subtree while the wave walks it for other lanes.  Lanes without a face
// (live = false) take no node.  All lanes of the wave must call this together.
#pragma once
#include "tp_internal.h"
#include "tp_solver.h"   // wave_sum: a wave-wide sum in a fixed order

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tp {

// Block lists of the block cluster tree, built on the device (tp_bh.hip): one level of the
// breadth-first split per launch_bct_expand (pairs of nodes of one depth as (I << 32 | J);
// admissible blocks appended to far at cnt[0], exact leaf blocks (as leaf indices) to near
// at cnt[1], the next level's pairs to next at cnt[2]; the caller sizes far and near for
// n more entries and next for 4n), then launch_bct_sort_csr turns a list into CSR rows
// (sorted by row and column; off [rows + 1], col [n]).
size_t bct_sort_temp_bytes(int64_t n);
// rec [M][8] (64-byte aligned): per node lo, hi, r^2, a_I, written by launch_bct_nodes.
hipError_t launch_bct_nodes(const BhBuffers& b, int64_t M, double* rec, hipStream_t s);
hipError_t launch_bct_expand(const double* rec, int64_t P, double chi, const uint64_t* cur, int64_t n, uint64_t* far,
                             uint64_t* near, uint64_t* next, unsigned long long* cnt, hipStream_t s);
hipError_t launch_bct_sort_csr(const uint64_t* keys, uint64_t* sorted, int64_t n, void* tmp, size_t tmp_bytes,
                               int64_t rows, int32_t* off, int32_t* col, hipStream_t s);

// The walk itself: act(node, took) is called on every lane at every node the wave visits,
// with took = 1 when the node is admissible for the lane, 2 when it is a leaf the lane sums
// exactly, 0 otherwise (the call is uniform across the wave, so act may use cross-lane
// operations).
template <class Adm, class Act>
__device__ __forceinline__ void wave_walk_act(const double* __restrict__ na, int64_t P, bool live, Adm&& adm,
                                              Act&& act)
{
    int node = 1;
    int skip = live ? 0 : 1;   // root of the subtree this lane skips (0: none; 1: the whole tree)
    for (;;) {
        node = __builtin_amdgcn_readfirstlane(node);   // the same on every lane
        if (skip) {
            const int dn = 31 - __builtin_clz((unsigned)node), ds = 31 - __builtin_clz((unsigned)skip);
            if (dn < ds || (node >> (dn - ds)) != skip) skip = 0;   // left the skipped subtree
        }
        bool down = false;
        int took = 0;
        if (!skip && na[node] > 0.0) {
            if (adm(node)) {
                took = 1;
                skip = node;
            } else if (node >= P) {
                took = 2;
                skip = node;
            } else {
                down = true;
            }
        }
        act(node, took);
        if (__ballot(down) != 0ull) {
            node = 2 * node;
            continue;
        }
        while (node & 1) node >>= 1;   // climb out of right children (and the root)
        if (node == 0) break;
        node += 1;                     // right sibling
    }
}

// Add this lane's far and near term counts to counts[0], counts[1]: summed across the wave
// first, one atomic addition per wave.  All lanes of the wave must call this together.
__device__ __forceinline__ void wave_count_terms(unsigned long long* counts, unsigned long long nfar,
                                                 unsigned long long nnear)
{
    for (int o = 32; o > 0; o >>= 1) {
        nfar += __shfl_xor(nfar, o, 64);
        nnear += __shfl_xor(nnear, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (nfar) atomicAdd(&counts[0], nfar);
        if (nnear) atomicAdd(&counts[1], nnear);
    }
}

template <class Adm, class Far, class Near>
__device__ __forceinline__ void wave_walk(const double* __restrict__ na, int64_t P, bool live, Adm&& adm, Far&& far,
                                          Near&& near)
{
    wave_walk_act(na, P, live, adm, [&](int node, int took) {
        if (took == 1) far(node);
        else if (took == 2) near(node);
    });
}

}  // namespace tp
