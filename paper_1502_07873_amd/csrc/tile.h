// Tile bookkeeping shared by the tiled stencil kernels: the XCD-aware block
// order, cross-lane neighbour moves and the tile decode.
#pragma once

#include <hip/hip_runtime.h>

#include "ce.h"
#include "internal.h"

namespace eig {

namespace {

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that the
// tiles a given XCD works on at one time are contiguous (same solve, shared
// halos in that XCD's L2).  A bijection on [0, n) for any n.
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int x = b & 7, j = b >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + j;
}

// Value held by lane-1 (lane 0 receives `edge`) and by lane+1 (lane 63
// receives `edge`).  DPP wave shifts keep the old value in the lane whose
// source is outside the wavefront.
__device__ __forceinline__ float from_left(float x, float edge) {
    return __int_as_float(__builtin_amdgcn_update_dpp(
        __float_as_int(edge), __float_as_int(x), 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float x, float edge) {
    return __int_as_float(__builtin_amdgcn_update_dpp(
        __float_as_int(edge), __float_as_int(x), 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// Wave-uniform tile decode: tile entry = (solve, strip << 16 | chunk).
struct TileInfo {
    const SolveDesc* d;
    int m, x0, kb, ke;
};

__device__ __forceinline__ bool decode_tile(const SolveDesc* descs, const int2* tiles,
                                            int ntiles, int step, int cols, int rows,
                                            TileInfo& t) {
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return false;
    const int2 te = tiles[tile];
    const int sidx = __builtin_amdgcn_readfirstlane(te.x);
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    t.d = descs + sidx;
    t.m = step - t.d->start;
    if (t.m < 0 || t.m >= t.d->nsteps) return false;
    t.x0 = (sc >> 16) * cols;
    t.kb = (sc & 0xffff) * rows;
    t.ke = min(t.kb + rows, t.d->nz - 1);  // rows [kb, ke) are free rows
    return true;
}

// True if this wave's tile is an edge tile (absorbing edge nodes, ce.h):
// the wave updates them and the kernel returns.
__device__ __forceinline__ bool edge_wave(const SolveDesc* descs, const int2* tiles,
                                          int ntiles, int step) {
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return false;
    return ce_edge_tile(descs, tiles[tile], step, threadIdx.x & 63);
}

}  // namespace

}  // namespace eig
