// Propagation-step kernels for gfx950 (one lane per fluid node).
//
// PDF storage, tile-major structure of arrays: node n = 64 t + l keeps its
// direction q at element (19 t + q) * 64 + l. A 64-node wavefront tile thus
// loads and stores each direction as one coalesced 64-element segment, and
// the 19 segments of a tile are adjacent: a wave streams one contiguous
// block instead of 19 distant streams (the 19 "arrays" of Sect. 4.3 become
// 19 rows of one tile). Neighbour gathers of the odd step stay contiguous
// inside runs, which is what reduced indirect addressing exploits.
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
//  * Per-direction RIA: the same rule kept separately for each direction
//    (IndexRIADir below), for lattices where the joint runs are short.
#pragma once

#include "d3q19.hpp"

namespace lbm {

constexpr int kBlock = 256;
static_assert(kBlock == kGroupNodes, "a workgroup covers one schedule block");

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, so in
// plain order neighbouring tiles run on different XCDs and the cache lines
// they share (partial lines of the scattered stores, gathered lines) meet in
// no common L2. With chunks of K > 0 workgroup tiles (256 nodes each), the
// tiles are cut into chunks of K consecutive tiles, and XCD x (the XCD of
// workgroup b is b mod 8) takes chunks x, x + 8, x + 16, ... in turn.
// Neighbouring tiles then share an L2, while the 8 XCDs still sweep one
// region of memory together. The grid must be a multiple of 8K (the extra
// workgroups find no nodes and return).
__device__ __forceinline__ int64_t tile_index(int chunk) {
  if (chunk <= 0) return blockIdx.x;
  const int64_t k = chunk, x = blockIdx.x & 7, seq = blockIdx.x >> 3;
  return ((seq / k) * 8 + x) * k + seq % k;
}

// A workgroup's tile from an explicit schedule (host-validated: every tile
// once, -1 for an empty slot), or from the chunked order without one.
__device__ __forceinline__ int64_t scheduled_tile(int chunk, const int32_t* __restrict__ sched) {
  return sched ? (int64_t)sched[blockIdx.x] : tile_index(chunk);
}

// ---------------------------------------------------------------- indices --

struct IndexIA {
  const int32_t* __restrict__ adj;
  int64_t lda;  // 18 * lda may exceed 2^31

  __device__ __forceinline__ void get(int32_t n, int32_t (&a)[18]) const {
#pragma unroll
    for (int q = 0; q < 18; ++q) a[q] = __builtin_nontemporal_load(adj + q * lda + n);
  }
};

struct IndexRIA {
  const int32_t* __restrict__ delta;
  const uint64_t* __restrict__ head_bits;
  const int32_t* __restrict__ run_base;
  int64_t ldr;  // 18 * ldr may exceed 2^31

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

// Per-direction RIA: the run rule applied to one direction at a time, so a
// run of direction q only breaks where the entries of q stop shifting by one.
// On fragmented porous media a node then rarely needs fresh deltas for all 18
// directions: the tables hold 4 B per direction run plus 12 B per wave and
// direction, against 72 B per run of the joint encoding. Wave w reads its 18
// head words and 18 bases as wave-uniform values. Every lane then finds its
// run per direction with a popcount, and the 18 delta loads go out together;
// a direction whose run spans the whole wave reads one address in all lanes
// (one cache line). A scalar-load branch per direction for such directions
// measured slower: it serialises the loads of a wave.
struct IndexRIADir {
  const int32_t* __restrict__ delta;       // [RD]
  const uint64_t* __restrict__ head_bits;  // [W][18]
  const int32_t* __restrict__ run_base;    // [W][18]

  __device__ __forceinline__ void get(int32_t n, int32_t (&a)[18]) const {
    const int32_t w = __builtin_amdgcn_readfirstlane(n >> 6);
    const uint64_t* bw = head_bits + w * 18;
    const int32_t* rw = run_base + w * 18;
    const int lane = n & 63;
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    int32_t d[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) d[q] = delta[rw[q] + __popcll(bw[q] & upto)];
#pragma unroll
    for (int q = 0; q < 18; ++q) a[q] = d[q] == INT32_MIN ? -1 : n + d[q];
  }
};

// Slots are element offsets into the grid, of type Off: int32_t while the
// grid holds at most 2^31 - 1 elements (19 * ldf, lattices of up to
// 113 M nodes), int64_t beyond, so that one grid can fill the device. The
// 32-bit form needs no 64-bit integer arithmetic per slot; the host takes
// it whenever the grid allows. Node indices stay 32-bit (N < 2^31). Per
// lane a slot costs a compare, two selects and a few integer operations,
// with no branch.
constexpr int32_t kTile = 64;

// Offset of direction 0 of node m; direction q lies q * 64 elements further.
template <class Off = int32_t>
__device__ __forceinline__ Off node_base(int32_t m) {
  return (Off)(m & ~(kTile - 1)) * Q + (m & (kTile - 1));
}

template <class Off = int32_t>
__device__ __forceinline__ Off pdf_slot(int q, int32_t m) { return node_base<Off>(m) + q * kTile; }

// AA odd-step slot of f_q for node n: L_q(n) = (qbar at a_q(n)) or (q at n).
template <class Off = int32_t>
__device__ __forceinline__ Off aa_slot(int q, int32_t n, const int32_t (&a)[18]) {
  if (q == 0) return node_base<Off>(n);
  const int32_t an = a[q - 1];
  const bool fluid = an >= 0;
  const int32_t m = fluid ? an : n;
  return node_base<Off>(m) + (fluid ? kOpp[q] : q) * kTile;
}

// OS-NT pull slot of f_q for node n: (q at a_q(n)) or (qbar at n).
template <class Off = int32_t>
__device__ __forceinline__ Off pull_slot(int q, int32_t n, const int32_t (&a)[18]) {
  if (q == 0) return node_base<Off>(n);
  const int32_t an = a[q - 1];
  const bool fluid = an >= 0;
  const int32_t m = fluid ? an : n;
  return node_base<Off>(m) + (fluid ? q : kOpp[q]) * kTile;
}

// ------------------------------------------------------------- step kernels --
// S is the storage type: double (FP64 arithmetic in the oracle's order),
// float or _Float16 (deviation storage, FP32 arithmetic). TRT selects the
// collision (BGK or TRT) at compile time, so each kernel only holds the
// registers of its own operator. Off is the slot type (above).

template <class S, bool TRT, class Off>
__global__ void __launch_bounds__(kBlock)
aa_even(S* __restrict__ F, int32_t N, Collision c, int chunk) {
  const int64_t n64 = tile_index(chunk) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  S* Fn = F + node_base<Off>(n);
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = __builtin_nontemporal_load(Fn + q * kTile);
  Prec<S>::template collide<TRT>(f, c);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(f[q], Fn + kOpp[q] * kTile);
}

// Minimum waves per SIMD the compiler must leave room for in the odd step
// (1: no constraint). The FP16 odd step otherwise takes 81 VGPRs (5 waves);
// asked for 6 it fits in 67 without spilling and runs 7 waves, which hides
// more of its gather latency (2-3 % faster on the sphere pack). FP32 gains
// nothing, and FP64 would spill.
template <class S> struct OddWaves { static constexpr int value = sizeof(S) == 2 ? 6 : 1; };

template <class S, class Idx, bool TRT, class Off>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(OddWaves<S>::value)))
aa_odd(S* __restrict__ F, int32_t N, Idx idx, Collision c, int chunk, const int32_t* __restrict__ sched) {
  const int64_t tile = scheduled_tile(chunk, sched);
  if (tile < 0) return;
  const int64_t n64 = tile * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int32_t a[18];
  idx.get(n, a);
  Off slot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) slot[q] = aa_slot<Off>(q, n, a);
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = F[slot[q]];
  Prec<S>::template collide<TRT>(f, c);
  // f*_q goes where f_qbar came from
#pragma unroll
  for (int q = 0; q < Q; ++q) F[slot[kOpp[q]]] = f[q];
}

template <class S, class Idx, bool TRT, class Off>
__global__ void __launch_bounds__(kBlock)
osnt(const S* __restrict__ G, S* __restrict__ H, int32_t N, Idx idx, Collision c, int chunk) {
  const int64_t n64 = tile_index(chunk) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int32_t a[18];
  idx.get(n, a);
  Off slot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) slot[q] = pull_slot<Off>(q, n, a);
  S f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = G[slot[q]];
  Prec<S>::template collide<TRT>(f, c);
  S* Hn = H + node_base<Off>(n);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(f[q], Hn + q * kTile);
}

}  // namespace lbm
