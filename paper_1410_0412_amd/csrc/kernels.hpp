// Propagation-step kernels for gfx950 (one lane per fluid node).
//
// PDF storage: F[q*ldf + n], 19 direction streams of one element per fluid
// node (structure of arrays), ldf a multiple of 64 so that every stream of a
// 64-node wavefront tile starts on its own aligned segment. A wavefront of 64
// consecutive nodes therefore loads and stores each direction as one
// contiguous 64-element segment whenever the nodes lie in one run, which is
// what reduced indirect addressing exploits.
//
// Propagation patterns (Sect. 4):
//  * AA, even step (direct): read (q, n), collide, write f*_q to (qbar, n).
//  * AA, odd step (indirect): read f_q from L_q(n) = (qbar, a_q(n)), or
//    (q, n) when the upstream site is solid (halfway bounce-back); collide;
//    write f*_q to L_qbar(n), the slot f_qbar came from. L is a bijection on
//    slots, so the step runs in place without races.
//  * OS-NT (pull, two grids): read f_q from (q, a_q(n)) of grid G, or
//    (qbar, n) for a solid upstream site; collide; write (q, n) of grid H.
// a_q(n) is the adjacency entry (upstream node of n along c_q, or -1).
//
// Neighbour resolution:
//  * IA: 18 int32 loads of the adjacency list per node (Sect. 4, D_idx).
//  * RIA (Sect. 4.1): runs of nodes whose entries are those of the previous
//    node shifted by one share one table column: a_q(n) = n + delta_q(run).
//    The run of a lane comes from the wave's head bitmap with a popcount, so
//    no per-node run index is stored. When a whole 64-node wave lies in one
//    run, the 18 deltas are wave-uniform and are fetched with scalar loads:
//    no vector index load is issued at all (the GPU counterpart of the
//    partial vectorization of Sect. 4.2).
#pragma once

#include "d3q19.hpp"

namespace lbm {

constexpr int kBlock = 256;

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; with
// remapping, each XCD sweeps one contiguous range of tiles, so the partial
// cache lines shared by neighbouring tiles stay in that XCD's L2.
__device__ __forceinline__ int64_t tile_index(int remap) {
  if (!remap) return blockIdx.x;
  const int64_t per = gridDim.x >> 3;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// ---------------------------------------------------------------- indices --

struct IndexIA {
  const int32_t* __restrict__ adj;
  int32_t lda;

  __device__ __forceinline__ void get(int32_t n, int32_t (&a)[18]) const {
#pragma unroll
    for (int q = 0; q < 18; ++q) a[q] = __builtin_nontemporal_load(adj + q * lda + n);
  }
};

struct IndexRIA {
  const int32_t* __restrict__ delta;
  const uint64_t* __restrict__ head_bits;
  const int32_t* __restrict__ run_base;
  int32_t ldr;

  __device__ __forceinline__ void get(int32_t n, int32_t (&a)[18]) const {
    // all lanes of the wave hold nodes 64w .. 64w+63
    const int32_t w = __builtin_amdgcn_readfirstlane(n >> 6);
    const uint64_t bits = head_bits[w];
    const int32_t base = run_base[w];
    if ((bits >> 1) == 0) {
      // one run covers the wave: wave-uniform deltas via scalar loads
      const int32_t r = __builtin_amdgcn_readfirstlane(base + (int32_t)(bits & 1));
#pragma unroll
      for (int q = 0; q < 18; ++q) {
        const int32_t d = delta[q * ldr + r];
        a[q] = d == INT32_MIN ? -1 : n + d;
      }
    } else {
      const int lane = n & 63;
      const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      const int32_t r = base + __popcll(bits & upto);
#pragma unroll
      for (int q = 0; q < 18; ++q) {
        const int32_t d = delta[q * ldr + r];
        a[q] = d == INT32_MIN ? -1 : n + d;
      }
    }
  }
};

// Slots are 32-bit element offsets into the grid (the host guarantees
// 19 * ldf < 2^31). Stream offsets q * ldf are wave-uniform and kept in
// scalar registers; per lane a slot costs one compare, two selects and one
// add, with no branch.
__device__ __forceinline__ int32_t stream_offset(int q, int32_t ldf) {
  return __builtin_amdgcn_readfirstlane(q * ldf);
}

__device__ __forceinline__ int32_t select_slot(int32_t an, int32_t n, int32_t base_fluid,
                                               int32_t base_wall) {
  const bool fluid = an >= 0;
  const int32_t idx = fluid ? an : n;
  const int32_t base = fluid ? base_fluid : base_wall;
  return base + idx;
}

// AA odd-step slot of f_q for node n: L_q(n).
__device__ __forceinline__ int32_t aa_slot(int q, int32_t n, const int32_t (&a)[18], int32_t ldf) {
  if (q == 0) return n;
  return select_slot(a[q - 1], n, stream_offset(kOpp[q], ldf), stream_offset(q, ldf));
}

// OS-NT pull slot of f_q for node n.
__device__ __forceinline__ int32_t pull_slot(int q, int32_t n, const int32_t (&a)[18], int32_t ldf) {
  if (q == 0) return n;
  return select_slot(a[q - 1], n, stream_offset(q, ldf), stream_offset(kOpp[q], ldf));
}

// ------------------------------------------------------------- step kernels --
// S is the storage type: double (FP64 arithmetic in the oracle's order),
// float or _Float16 (deviation storage, FP32 arithmetic). TRT selects the
// collision (BGK or TRT) at compile time, so each kernel only holds the
// registers of its own operator.

template <class S, bool TRT>
__global__ void __launch_bounds__(kBlock)
aa_even(S* __restrict__ F, int32_t N, int32_t ldf, Collision c, int remap) {
  const int64_t n64 = tile_index(remap) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = __builtin_nontemporal_load(F + (stream_offset(q, ldf) + n));
  Prec<S>::template collide<TRT>(f, c);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(f[q], F + (stream_offset(kOpp[q], ldf) + n));
}

template <class S, class Idx, bool TRT>
__global__ void __launch_bounds__(kBlock)
aa_odd(S* __restrict__ F, int32_t N, int32_t ldf, Idx idx, Collision c, int remap) {
  const int64_t n64 = tile_index(remap) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int32_t a[18];
  idx.get(n, a);
  int32_t slot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) slot[q] = aa_slot(q, n, a, ldf);
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = F[slot[q]];
  Prec<S>::template collide<TRT>(f, c);
  // f*_q goes where f_qbar came from
#pragma unroll
  for (int q = 0; q < Q; ++q) F[slot[kOpp[q]]] = f[q];
}

template <class S, class Idx, bool TRT>
__global__ void __launch_bounds__(kBlock)
osnt(const S* __restrict__ G, S* __restrict__ H, int32_t N, int32_t ldf, Idx idx, Collision c,
     int remap) {
  const int64_t n64 = tile_index(remap) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int32_t a[18];
  idx.get(n, a);
  int32_t slot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) slot[q] = pull_slot(q, n, a, ldf);
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = G[slot[q]];
  Prec<S>::template collide<TRT>(f, c);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(f[q], H + (stream_offset(q, ldf) + n));
}

}  // namespace lbm
