// Device solver and bandwidth micro-benchmarks behind the C ABI of
// include/lbm_sparse.h: initialisation, time stepping (AA or OS-NT, with
// adjacency list, RIA wave tables or per-direction RIA tables), macroscopic
// moments with deterministic FP64 reductions, and PDF export / import in
// natural order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "adjoint.hpp"
#include "kernels.hpp"

using namespace lbm;

struct lbm_solver {
  lbm_params p;
  lbm_buffers b;
  double* ws = nullptr;
  int64_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int64_t t = 0;
  int cur = 0;     // OS-NT: grid that holds f*(t-1)
  bool remap = true;  // XCD-aware tile order for the indirect steps
  bool lds_ready = false;  // occupancy reservations below computed
  unsigned even_lds = 0, pull_lds = 0;  // LDS bytes reserved per workgroup
  bool trt = false;
  Collision c;
  const int32_t* odd_sched = nullptr;  // device schedule of the AA odd step, or null
  int64_t odd_sched_len = 0;
};

namespace {

constexpr int kRedBlocks = 1024;  // fixed grid of the reduction: deterministic sums

// Which slots hold f(t) for node n: natural (AA at even t), L (AA at odd t)
// or the pull map P (OS-NT). The kernels outside the time loop take 64-bit
// slots for every lattice.
enum Layout : int { kNatural = 0, kAAOdd = 1, kPull = 2 };

template <class Idx>
__device__ __forceinline__ void state_slots(int layout, int32_t n, const Idx& idx, int64_t (&s)[Q]) {
  if (layout == kNatural) {
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = pdf_slot<int64_t>(q, n);
    return;
  }
  int32_t a[18];
  idx.get(n, a);
  if (layout == kAAOdd) {
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = aa_slot<int64_t>(q, n, a);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = pull_slot<int64_t>(q, n, a);
  }
}

template <class S, class Idx>
__global__ void __launch_bounds__(kBlock)
init_eq(S* __restrict__ F, int32_t N, Idx idx, int layout,
        const double* __restrict__ rho, const double* __restrict__ u, Collision c) {
  const int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  const double r = rho ? rho[n] : c.rho0;
  const double ux = u ? u[n] : 0.0, uy = u ? u[(int64_t)N + n] : 0.0, uz = u ? u[2 * (int64_t)N + n] : 0.0;
  double v[Q];
  if constexpr (Prec<S>::kDeviation) {
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = equilibrium_dev_f64(q, r, c.rho0, ux, uy, uz);
  } else {
    equilibrium_f64(r, ux, uy, uz, v);
  }
  int64_t s[Q];
  state_slots(layout, n, idx, s);
#pragma unroll
  for (int q = 0; q < Q; ++q) F[s[q]] = Prec<S>::from64(q, v[q], c);
}

// f(t) in natural order, FP64.
template <class S, class Idx>
__global__ void __launch_bounds__(kBlock)
gather_pdfs(const S* __restrict__ F, int32_t N, Idx idx, int layout, Collision c,
            double* __restrict__ out) {
  const int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int64_t s[Q];
  state_slots(layout, n, idx, s);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double v = Prec<S>::value64(q, F[s[q]], c);
    out[(int64_t)q * N + n] = Prec<S>::kDeviation ? kW[q] * c.rho0 + v : v;
  }
}

template <class S, class Idx>
__global__ void __launch_bounds__(kBlock)
scatter_pdfs(S* __restrict__ F, int32_t N, Idx idx, int layout, Collision c,
             const double* __restrict__ in) {
  const int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int64_t s[Q];
  state_slots(layout, n, idx, s);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double f = in[(int64_t)q * N + n];
    F[s[q]] = Prec<S>::from64(q, Prec<S>::kDeviation ? f - kW[q] * c.rho0 : f, c);
  }
}

// rho, u = j / rho of f(t), plus per-block partial sums of rho and j, all in
// FP64. FP64 storage: the oracle's folds over f. Deviation storage: folds
// over the deviations, rho = rho0 + sum_q d_q.
template <class S, class Idx>
__global__ void __launch_bounds__(kBlock)
moments(const S* __restrict__ F, int32_t N, Idx idx, int layout, Collision c,
        double* __restrict__ rho_out, double* __restrict__ u_out, double* __restrict__ partial) {
  __shared__ double red[4][kBlock];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x; n64 < N;
       n64 += (int64_t)gridDim.x * kBlock) {
    const int32_t n = (int32_t)n64;
    int64_t s[Q];
    state_slots(layout, n, idx, s);
    double f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = Prec<S>::value64(q, F[s[q]], c);
    const double rho = Prec<S>::kDeviation ? c.rho0 + density(f) : density(f);
    const double jx = momentum<0>(f), jy = momentum<1>(f), jz = momentum<2>(f);
    if (rho_out) rho_out[n] = rho;
    if (u_out) {
      u_out[n] = jx / rho;
      u_out[(int64_t)N + n] = jy / rho;
      u_out[2 * (int64_t)N + n] = jz / rho;
    }
    acc[0] = acc[0] + rho;
    acc[1] = acc[1] + jx;
    acc[2] = acc[2] + jy;
    acc[3] = acc[3] + jz;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = red[k][threadIdx.x] + red[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Partial sums of w_n j_axis(n) of f(t) (FP64).
template <class S, class Idx>
__global__ void __launch_bounds__(kBlock)
weighted_momentum(const S* __restrict__ F, int32_t N, Idx idx, int layout, Collision c,
                  const double* __restrict__ w, int axis, double* __restrict__ partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x; n64 < N;
       n64 += (int64_t)gridDim.x * kBlock) {
    const int32_t n = (int32_t)n64;
    int64_t s[Q];
    state_slots(layout, n, idx, s);
    double f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = Prec<S>::value64(q, F[s[q]], c);
    const double j = axis == 0 ? momentum<0>(f) : (axis == 1 ? momentum<1>(f) : momentum<2>(f));
    acc = acc + w[n] * j;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + k];
    __syncthreads();
  }
  // same partial layout as the moments kernel: 4 doubles per block
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = threadIdx.x == 0 ? red[0] : 0.0;
}

__global__ void __launch_bounds__(kBlock)
finish_totals(const double* __restrict__ partial, int nparts, double* __restrict__ totals) {
  __shared__ double red[4][kBlock];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = acc[k] + partial[i * 4 + k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = red[k][threadIdx.x] + red[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) totals[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------- micro-benchmarks ----

typedef double vec2d __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(kBlock)
bench_copy(const vec2d* __restrict__ src, vec2d* __restrict__ dst, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n2) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void __launch_bounds__(kBlock)
bench_copy_tail(const double* __restrict__ src, double* __restrict__ dst, int64_t lo, int64_t n) {
  const int64_t i = lo + (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void __launch_bounds__(kBlock)
bench_cnt19(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = __builtin_nontemporal_load(src + q * ld + i);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q], dst + q * ld + i);
}

__global__ void __launch_bounds__(kBlock)
bench_u19(double* __restrict__ F, int64_t n, int64_t ld, double s) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = __builtin_nontemporal_load(F + q * ld + i);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q] * s, F + q * ld + i);
}

// The same update in the tile-major layout of the PDF grid, workgroups in
// plain or chunked XCD-aware tile order (chunk > 0, as the step kernels).
__global__ void __launch_bounds__(kBlock)
bench_u19_tiles(double* __restrict__ F, int64_t n, double s, int chunk) {
  const int64_t i = tile_index(chunk) * kBlock + threadIdx.x;
  if (i >= n) return;
  double* Fi = F + (i & ~(int64_t)(kTile - 1)) * Q + (i & (kTile - 1));
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = __builtin_nontemporal_load(Fi + q * kTile);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q] * s, Fi + q * kTile);
}

__global__ void __launch_bounds__(kBlock)
bench_cnt19_tiles(const double* __restrict__ src, double* __restrict__ dst, int64_t n, int chunk) {
  const int64_t i = tile_index(chunk) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t o = (i & ~(int64_t)(kTile - 1)) * Q + (i & (kTile - 1));
  double v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = __builtin_nontemporal_load(src + o + q * kTile);
#pragma unroll
  for (int q = 0; q < Q; ++q) __builtin_nontemporal_store(v[q], dst + o + q * kTile);
}

__global__ void __launch_bounds__(kBlock)
bench_u1(double* __restrict__ F, int64_t n, double s) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(F + i) * s, F + i);
}

// ---------------------------------------------------------------- host ----

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int device_status(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

IndexIA index_ia(const lbm_solver* s) { return IndexIA{s->b.adj, s->p.lda}; }
IndexRIA index_ria(const lbm_solver* s) {
  return IndexRIA{s->b.run_delta, s->b.head_bits, s->b.run_base, s->p.ldr};
}
IndexRIADir index_ria_dir(const lbm_solver* s) {
  return IndexRIADir{s->b.run_delta, s->b.head_bits, s->b.run_base};
}

// Call go(idx) with the neighbour index source of the solver.
template <class Go>
void with_index(const lbm_solver* s, Go&& go) {
  switch (s->p.ria) {
    case LBM_INDEX_RUNS: go(index_ria(s)); break;
    case LBM_INDEX_DIRECTION_RUNS: go(index_ria_dir(s)); break;
    default: go(index_ia(s)); break;
  }
}

// Call go(Off{}) with the slot type of the time-step kernels: 32-bit while
// the grid's 19 * ldf elements fit in 31 bits, 64-bit for larger grids or
// when the caller asks for them.
template <class Go>
void with_slots(const lbm_solver* s, Go&& go) {
  if ((s->p.flags & LBM_FLAG_WIDE_SLOTS) || (int64_t)Q * s->p.ldf > (int64_t)INT32_MAX)
    go(int64_t{});
  else
    go(int32_t{});
}

// Layout of f(t) in the current grid.
int current_layout(const lbm_solver* s) {
  if (s->p.pattern == LBM_PATTERN_OSNT) return kPull;
  return (s->t % 2 == 0) ? kNatural : kAAOdd;
}

void* current_grid(const lbm_solver* s) {
  return s->b.pdf[s->p.pattern == LBM_PATTERN_OSNT ? s->cur : 0];
}

// Call fn(S*, idx) with the storage type and index source of the solver.
template <class Fn>
void dispatch(const lbm_solver* s, void* grid, Fn&& fn) {
  auto with_idx = [&](auto* typed) { with_index(s, [&](auto idx) { fn(typed, idx); }); };
  switch (s->p.precision) {
    case LBM_F64: with_idx((double*)grid); break;
    case LBM_F32: with_idx((float*)grid); break;
    default: with_idx((_Float16*)grid); break;
  }
}

// Chunks of the XCD-aware tile order (workgroups of 256 nodes), measured on
// the sphere pack, the foam and the channel: 32-64 for the AA odd step,
// 8-32 for OS-NT; smaller chunks split neighbours, larger ones spread the
// XCDs over distant regions of memory. The even step shares no lines between
// tiles; it takes the odd step's order, which measured 0-2 % faster than
// plain order.
constexpr int kOddChunk = 64;
constexpr int kEvenChunk = 64;
constexpr int kPullChunk = 16;

// Occupancy caps (workgroups per CU; 0 = as many as the registers allow),
// measured per storage precision. The streaming even step in FP64 and FP32
// runs fastest with 2 workgroups (8 waves) per CU: fewer requests in flight
// keep the DRAM accesses in order (FP64: -2 % of its time on the sphere pack,
// -8 % on the 384^3 foam; FP32 on the foam: -13 %). In FP16 a wave moves a
// quarter of the bytes and the cap costs 25 %. OS-NT in FP64 runs best with
// 5. The odd step needs all the concurrency it gets for its gathers. The cap
// is an LDS reservation in the launch; the kernels use no LDS.
constexpr int kEvenWgsPerCu[3] = {2, 2, 0};  // LBM_F64, LBM_F32, LBM_F16
constexpr int kPullWgsPerCu[3] = {5, 0, 0};

// LDS bytes per workgroup that allow exactly `wgs` workgroups per CU, or 0
// (no cap) if the device limits cannot express it.
unsigned lds_for(int per_cu, int per_block, int wgs) {
  if (per_cu <= 0 || per_block <= 0 || wgs <= 0) return 0;
  const int bytes = std::min(per_cu / wgs, per_block);
  return (bytes > 0 && per_cu / bytes == wgs) ? (unsigned)bytes : 0;
}

// LDS bytes per workgroup that cap a launch on the current device at `wgs`
// workgroups per CU (0: no cap).
unsigned lds_for_device(int wgs) {
  int dev = 0, per_cu = 0, per_block = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0;
  return lds_for(per_cu, per_block, wgs);
}

void init_occupancy(lbm_solver* s) {
  int dev = 0, per_cu = 0, per_block = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    per_cu = per_block = 0;  // no caps
  }
  const int k = s->p.precision;  // validated: LBM_F64, LBM_F32 or LBM_F16
  s->even_lds = lds_for(per_cu, per_block, kEvenWgsPerCu[k]);
  s->pull_lds = lds_for(per_cu, per_block, kPullWgsPerCu[k]);
  s->lds_ready = true;
}

// Grid of a launch in chunked tile order: a multiple of 8 * chunk.
inline unsigned chunked_grid(unsigned tiles, int chunk) {
  const unsigned m = 8u * (unsigned)chunk;
  return chunk > 0 ? (tiles + m - 1) / m * m : tiles;
}

template <bool TRT, class Off>
void launch_step_op(lbm_solver* s, int32_t N) {
  const unsigned tiles = grid_for(N);
  const dim3 b(kBlock);
  if (!s->lds_ready) init_occupancy(s);
  if (s->p.pattern == LBM_PATTERN_AA) {
    if (s->t % 2 == 0) {
      dispatch(s, s->b.pdf[0], [&](auto* F, auto) {
        using S = std::remove_pointer_t<decltype(F)>;
        const int chunk = s->remap ? kEvenChunk : 0;
        hipLaunchKernelGGL((aa_even<S, TRT, Off>), dim3(chunked_grid(tiles, chunk)), b, s->even_lds, s->stream,
                           F, N, s->c, chunk);
      });
    } else {
      // the scattered stores of the odd step share partial lines between
      // neighbouring tiles: keep neighbours on one XCD
      const int chunk = s->remap ? kOddChunk : 0;
      const unsigned grid = s->odd_sched ? (unsigned)s->odd_sched_len : chunked_grid(tiles, chunk);
      dispatch(s, s->b.pdf[0], [&](auto* F, auto idx) {
        using S = std::remove_pointer_t<decltype(F)>;
        hipLaunchKernelGGL((aa_odd<S, decltype(idx), TRT, Off>), dim3(grid), b, 0, s->stream, F, N, idx, s->c,
                           chunk, s->odd_sched);
      });
    }
  } else {
    void* G = s->b.pdf[s->cur];
    void* H = s->b.pdf[1 - s->cur];
    const int chunk = s->remap ? kPullChunk : 0;
    dispatch(s, G, [&](auto* Gt, auto idx) {
      using S = std::remove_pointer_t<decltype(Gt)>;
      hipLaunchKernelGGL((osnt<S, decltype(idx), TRT, Off>), dim3(chunked_grid(tiles, chunk)), b, s->pull_lds,
                         s->stream, (const S*)Gt, (S*)H, N, idx, s->c, chunk);
    });
  }
}

// The partial-bounce-back step (AA, FP64, BGK); save != NULL also writes
// f(t) into save.
void launch_step_pbb(lbm_solver* s, int32_t N, double* save) {
  double* F = (double*)s->b.pdf[0];
  // the odd step's tile order (the even step of the PBB path shares it)
  const int chunk = s->remap ? kOddChunk : 0;
  const dim3 grid(chunked_grid(grid_for(N), chunk));
  auto go = [&](auto idx, auto off) {
    using I = decltype(idx);
    using Off = decltype(off);
    auto launch = [&](auto odd, auto keep) {
      hipLaunchKernelGGL((aa_step_pbb<I, decltype(odd)::value, decltype(keep)::value, Off>), grid, dim3(kBlock),
                         0, s->stream, F, N, idx, s->c, s->b.solid_frac, save, chunk);
    };
    const bool odd = s->t % 2 != 0;
    if (save)
      odd ? launch(std::true_type{}, std::true_type{}) : launch(std::false_type{}, std::true_type{});
    else
      odd ? launch(std::true_type{}, std::false_type{}) : launch(std::false_type{}, std::false_type{});
  };
  with_index(s, [&](auto idx) { with_slots(s, [&](auto off) { go(idx, off); }); });
}

int launch_step(lbm_solver* s) {
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N > 0 && s->b.solid_frac) {
    launch_step_pbb(s, N, nullptr);
  } else if (N > 0) {
    with_slots(s, [&](auto off) {
      using Off = decltype(off);
      if (s->trt)
        launch_step_op<true, Off>(s, N);
      else
        launch_step_op<false, Off>(s, N);
    });
  }
  if (s->p.pattern == LBM_PATTERN_OSNT) s->cur = 1 - s->cur;
  s->t += 1;
  return LBM_OK;
}

// Node and run indices are 32-bit, so no leading dimension needs more than
// 2^31 entries (N <= 2^31 - 65 rounds up to at most 2^31 - 64).
constexpr int64_t kMaxLd = (int64_t)1 << 31;

int validate(const lbm_params* p, const lbm_buffers* b) {
  if (!p || !b) return fail(LBM_EINVAL, "null params or buffers");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 1/2");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force[a])) return fail(LBM_EINVAL, "force must be finite");
  if (!std::isfinite(p->rho0) || !(p->rho0 > 0)) return fail(LBM_EINVAL, "rho0 must be positive");
  if (p->pattern != LBM_PATTERN_AA && p->pattern != LBM_PATTERN_OSNT)
    return fail(LBM_EINVAL, "unknown pattern %d", p->pattern);
  if (p->ria != LBM_INDEX_ADJ && p->ria != LBM_INDEX_RUNS && p->ria != LBM_INDEX_DIRECTION_RUNS)
    return fail(LBM_EINVAL, "ria must be 0, 1 or 2");
  if (p->precision != LBM_F64 && p->precision != LBM_F32 && p->precision != LBM_F16)
    return fail(LBM_EINVAL, "unknown precision %d", p->precision);
  if (p->flags & ~(LBM_FLAG_NO_XCD_REMAP | LBM_FLAG_WIDE_SLOTS))
    return fail(LBM_EINVAL, "unknown flags 0x%x", p->flags);
  if (p->f16_scale_log2 < -24 || p->f16_scale_log2 > 24) return fail(LBM_EINVAL, "f16_scale_log2 out of [-24, 24]");
  if (p->collision != LBM_BGK && p->collision != LBM_TRT) return fail(LBM_EINVAL, "unknown collision %d", p->collision);
  if (p->collision == LBM_TRT && !(p->trt_magic > 0 && std::isfinite(p->trt_magic)))
    return fail(LBM_EINVAL, "TRT needs a positive magic parameter");
  if (p->n_fluid < 0) return fail(LBM_EINVAL, "n_fluid < 0");
  if (p->n_fluid > INT32_MAX - 64) return fail(LBM_ERANGE, "n_fluid exceeds the int32 node index");
  if (p->ldf < p->n_fluid || p->ldf % 64 != 0) return fail(LBM_EINVAL, "ldf must be >= N and a multiple of 64");
  if (p->ldf > kMaxLd) return fail(LBM_ERANGE, "ldf exceeds 2^31");
  if (!b->pdf[0]) return fail(LBM_EINVAL, "pdf[0] is null");
  if (p->pattern == LBM_PATTERN_OSNT && !b->pdf[1]) return fail(LBM_EINVAL, "OS-NT needs pdf[1]");
  if (b->solid_frac && (p->pattern != LBM_PATTERN_AA || p->precision != LBM_F64 || p->collision != LBM_BGK))
    return fail(LBM_EINVAL, "partial bounce-back needs the AA pattern, FP64 and BGK");
  if (p->ria == LBM_INDEX_DIRECTION_RUNS) {
    if (p->n_runs < 0 || (p->n_fluid > 0 && p->n_runs < 18)) return fail(LBM_EINVAL, "n_runs invalid");
    if (p->n_runs > INT32_MAX) return fail(LBM_ERANGE, "per-direction run count exceeds int32");
    if (p->n_fluid > 0 && (!b->run_delta || !b->head_bits || !b->run_base))
      return fail(LBM_EINVAL, "per-direction RIA needs run_delta, head_bits and run_base");
  } else if (p->ria == LBM_INDEX_RUNS) {
    if (p->n_runs < 0 || (p->n_fluid > 0 && p->n_runs < 1)) return fail(LBM_EINVAL, "n_runs invalid");
    if (p->ldr < p->n_runs) return fail(LBM_EINVAL, "ldr < n_runs");
    if (p->ldr > kMaxLd) return fail(LBM_ERANGE, "ldr exceeds 2^31");
    if (p->n_fluid > 0 && (!b->run_delta || !b->head_bits || !b->run_base))
      return fail(LBM_EINVAL, "RIA needs run_delta, head_bits and run_base");
  } else {
    if (p->lda < p->n_fluid) return fail(LBM_EINVAL, "lda < n_fluid");
    if (p->lda > kMaxLd) return fail(LBM_ERANGE, "lda exceeds 2^31");
    if (p->n_fluid > 0 && !b->adj) return fail(LBM_EINVAL, "adjacency list is null");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_solver_workspace_bytes(const lbm_params* p, int64_t* bytes) {
  clear_error();
  if (!p || !bytes) return fail(LBM_EINVAL, "null pointer");
  *bytes = ((int64_t)kRedBlocks * 4 + 4) * sizeof(double);
  return LBM_OK;
}

int lbm_required_bytes(const lbm_params* p, int64_t* pdf_bytes_per_grid, int64_t* workspace_bytes) {
  clear_error();
  if (!p || !pdf_bytes_per_grid || !workspace_bytes) return fail(LBM_EINVAL, "null pointer");
  if (p->precision != LBM_F64 && p->precision != LBM_F32 && p->precision != LBM_F16)
    return fail(LBM_EINVAL, "unknown precision %d", p->precision);
  if (p->n_fluid < 0) return fail(LBM_EINVAL, "n_fluid < 0");
  if (p->n_fluid > INT32_MAX - 64) return fail(LBM_ERANGE, "n_fluid exceeds the int32 node index");
  const int64_t ldf = p->ldf == 0 ? (std::max<int64_t>(p->n_fluid, 1) + 63) / 64 * 64 : p->ldf;
  if (ldf < p->n_fluid || ldf % 64 != 0) return fail(LBM_EINVAL, "ldf must be 0, or >= N and a multiple of 64");
  if (ldf > kMaxLd) return fail(LBM_ERANGE, "ldf exceeds 2^31");
  const int64_t elem = p->precision == LBM_F64 ? 8 : (p->precision == LBM_F32 ? 4 : 2);
  *pdf_bytes_per_grid = Q * ldf * elem;
  return lbm_solver_workspace_bytes(p, workspace_bytes);
}

int lbm_solver_create(const lbm_params* p, const lbm_buffers* b, void* workspace,
                      int64_t workspace_bytes, void* hip_stream, lbm_solver** out) {
  clear_error();
  if (!out) return fail(LBM_EINVAL, "null out");
  *out = nullptr;
  int rc = validate(p, b);
  if (rc) return rc;
  int64_t need = 0;
  lbm_solver_workspace_bytes(p, &need);
  if (!workspace || workspace_bytes < need)
    return fail(LBM_EINVAL, "workspace must hold %lld bytes", (long long)need);
  lbm_solver* s = new (std::nothrow) lbm_solver;
  if (!s) return fail(LBM_ENOMEM, "out of host memory");
  s->p = *p;
  s->b = *b;
  s->ws = (double*)workspace;
  s->ws_bytes = workspace_bytes;
  s->stream = (hipStream_t)hip_stream;
  s->remap = (p->flags & LBM_FLAG_NO_XCD_REMAP) == 0;
  Collision& c = s->c;
  s->trt = p->collision == LBM_TRT;
  c.omega = 1.0 / p->tau;
  // Lambda = (1/w+ - 1/2)(1/w- - 1/2)  =>  w- = 1 / (Lambda / (tau - 1/2) + 1/2)
  c.omega_m = s->trt ? 1.0 / (p->trt_magic / (p->tau - 0.5) + 0.5) : c.omega;
  c.omega_m_f = (float)c.omega_m;
  for (int q = 0; q < Q; ++q) c.S[q] = (3.0 * kW[q]) * cdot<double>(q, p->force[0], p->force[1], p->force[2]);
  c.rho0 = p->rho0;
  c.omega_f = (float)c.omega;
  for (int q = 0; q < Q; ++q) c.S_f[q] = (float)c.S[q];
  c.rho0_f = (float)p->rho0;
  // FP16 stores d_q * 2^s / w_q: powers of two times 3, 18 or 36, exact in FP32
  const float two_s = std::ldexp(1.0f, p->f16_scale_log2);
  for (int q = 0; q < Q; ++q) {
    const float inv_w = q == 0 ? 3.0f : (q < 7 ? 18.0f : 36.0f);
    c.h_scale[q] = two_s * inv_w;
    c.h_unscale[q] = 1.0f / c.h_scale[q];
  }
  *out = s;
  return LBM_OK;
}

int lbm_solver_set_odd_schedule(lbm_solver* s, const int32_t* sched, int64_t len, int32_t* sched_device) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  if (!sched) {
    s->odd_sched = nullptr;
    s->odd_sched_len = 0;
    return LBM_OK;
  }
  if (s->p.pattern != LBM_PATTERN_AA) return fail(LBM_ESTATE, "only the AA pattern's odd step takes a schedule");
  if (!sched_device) return fail(LBM_EINVAL, "sched_device is null");
  if (len <= 0 || len % kXcds != 0 || len > (int64_t)INT32_MAX)
    return fail(LBM_EINVAL, "len must be a positive multiple of %d below 2^31", (int)kXcds);
  const int64_t G = (s->p.n_fluid + kGroupNodes - 1) / kGroupNodes;
  std::vector<uint8_t> seen((size_t)G, 0);
  int64_t blocks = 0;
  for (int64_t i = 0; i < len; ++i) {
    const int64_t g = sched[i];
    if (g == -1) continue;
    if (g < 0 || g >= G) return fail(LBM_EINVAL, "schedule entry %lld is %lld, outside [-1, %lld)", (long long)i,
                                     (long long)g, (long long)G);
    if (seen[(size_t)g]) return fail(LBM_EINVAL, "block %lld appears twice in the schedule", (long long)g);
    seen[(size_t)g] = 1;
    ++blocks;
  }
  if (blocks != G) return fail(LBM_EINVAL, "the schedule covers %lld of %lld blocks", (long long)blocks, (long long)G);
  if (hipMemcpyAsync(sched_device, sched, (size_t)len * sizeof(int32_t), hipMemcpyHostToDevice, s->stream) !=
          hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return device_status("set_odd_schedule (copy)");
  s->odd_sched = sched_device;
  s->odd_sched_len = len;
  return LBM_OK;
}

int lbm_solver_set_stream(lbm_solver* s, void* hip_stream) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  s->stream = (hipStream_t)hip_stream;
  return LBM_OK;
}

int lbm_solver_init_equilibrium(lbm_solver* s, const double* rho, const double* u) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  s->t = 0;
  s->cur = 0;
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N == 0) return LBM_OK;
  const int layout = s->p.pattern == LBM_PATTERN_OSNT ? kPull : kNatural;
  dispatch(s, s->b.pdf[0], [&](auto* F, auto idx) {
    using S = std::remove_pointer_t<decltype(F)>;
    hipLaunchKernelGGL((init_eq<S, decltype(idx)>), dim3(grid_for(N)), dim3(kBlock), 0, s->stream, F, N,
                       idx, layout, rho, u, s->c);
  });
  return device_status("init_equilibrium");
}

int lbm_solver_step(lbm_solver* s, int64_t n_steps) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  if (n_steps < 0) return fail(LBM_EINVAL, "n_steps < 0");
  for (int64_t i = 0; i < n_steps; ++i) launch_step(s);
  return device_status("step");
}

int lbm_solver_time(const lbm_solver* s, int64_t* t) {
  clear_error();
  if (!s || !t) return fail(LBM_EINVAL, "null pointer");
  *t = s->t;
  return LBM_OK;
}

namespace {
// The moments kernels with their partial sums in ws (kRedBlocks * 4 + 4
// doubles): per-block partials, then the four totals at ws + 4 * kRedBlocks,
// copied to totals if given. Synchronises the stream and checks that the
// totals are finite.
int moments_into(lbm_solver* s, double* ws, double* rho, double* u, double* totals) {
  const int32_t N = (int32_t)s->p.n_fluid;
  unsigned parts = 0;
  if (N > 0) {
    parts = std::min<unsigned>(grid_for(N), kRedBlocks);
    const int layout = current_layout(s);
    dispatch(s, current_grid(s), [&](auto* F, auto idx) {
      using S = std::remove_pointer_t<decltype(F)>;
      hipLaunchKernelGGL((moments<S, decltype(idx)>), dim3(parts), dim3(kBlock), 0, s->stream, (const S*)F,
                         N, idx, layout, s->c, rho, u, ws);
    });
  }
  // with no partials the finishing kernel writes zeros
  double* sums = ws + 4 * kRedBlocks;
  hipLaunchKernelGGL(finish_totals, dim3(1), dim3(kBlock), 0, s->stream, ws, (int)parts, sums);
  if (totals && hipMemcpyAsync(totals, sums, 4 * sizeof(double), hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
    return device_status("moments (copy)");
  double host[4] = {0.0, 0.0, 0.0, 0.0};
  if (hipMemcpyAsync(host, sums, sizeof host, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
    return device_status("moments (copy)");
  int rc = device_status("moments");
  if (rc) return rc;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return device_status("moments (sync)");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(host[k]))
      return fail(LBM_ERANGE, "non-finite %s total at t = %lld: the PDFs hold NaN or Inf",
                  k == 0 ? "mass" : "momentum", (long long)s->t);
  return LBM_OK;
}
}  // namespace

int lbm_solver_moments(lbm_solver* s, double* rho, double* u, double* totals) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  return moments_into(s, s->ws, rho, u, totals);
}

}  // extern "C"

namespace {
// Scratch of lbm_solver_moments_static: the partial sums of the moments
// kernels (kRedBlocks * 4 doubles) and the four totals, in device memory the
// library owns. Each device holds its own copy for the life of the process.
constexpr int kStaticScratchDoubles = kRedBlocks * 4 + 4;
__device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of the scratch array, looked
// up once per device (the array's name in host code is not that address).
int static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return device_status("moments_static (device)");
  if (dev >= kMaxDevices) return fail(LBM_ERANGE, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_EDEVICE, "moments_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_solver_moments_static(lbm_solver* s, double* rho, double* u, double* totals) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  // the moments kernels use at most kRedBlocks blocks for any lattice, so
  // their partial sums always fit; the check guards the constant
  int64_t need = 0;
  lbm_solver_workspace_bytes(&s->p, &need);
  if (need > (int64_t)sizeof(double) * kStaticScratchDoubles)
    return fail(LBM_ERANGE, "moments_static needs %lld bytes of scratch, the static array holds %lld",
                (long long)need, (long long)(sizeof(double) * kStaticScratchDoubles));
  double* ws = nullptr;
  int rc = static_scratch(&ws);
  if (rc) return rc;
  return moments_into(s, ws, rho, u, totals);
}

int lbm_solver_export_pdfs(lbm_solver* s, double* f) {
  clear_error();
  if (!s || !f) return fail(LBM_EINVAL, "null pointer");
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N > 0) {
    const int layout = current_layout(s);
    dispatch(s, current_grid(s), [&](auto* F, auto idx) {
      using S = std::remove_pointer_t<decltype(F)>;
      hipLaunchKernelGGL((gather_pdfs<S, decltype(idx)>), dim3(grid_for(N)), dim3(kBlock), 0, s->stream,
                         (const S*)F, N, idx, layout, s->c, f);
    });
  }
  int rc = device_status("export_pdfs");
  if (rc) return rc;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return device_status("export_pdfs (sync)");
  return LBM_OK;
}

int lbm_solver_import_pdfs(lbm_solver* s, const double* f, int64_t t) {
  clear_error();
  if (!s || !f) return fail(LBM_EINVAL, "null pointer");
  if (t < 0) return fail(LBM_EINVAL, "t < 0");
  s->t = t;
  s->cur = 0;
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N == 0) return LBM_OK;
  const int layout = current_layout(s);
  dispatch(s, current_grid(s), [&](auto* F, auto idx) {
    using S = std::remove_pointer_t<decltype(F)>;
    hipLaunchKernelGGL((scatter_pdfs<S, decltype(idx)>), dim3(grid_for(N)), dim3(kBlock), 0, s->stream, F,
                       N, idx, layout, s->c, f);
  });
  return device_status("import_pdfs");
}

int lbm_solver_set_time(lbm_solver* s, int64_t t) {
  clear_error();
  if (!s) return fail(LBM_EINVAL, "null solver");
  if (t < 0) return fail(LBM_EINVAL, "t < 0");
  if (s->p.pattern != LBM_PATTERN_AA) return fail(LBM_ESTATE, "set_time is defined for the AA pattern");
  s->t = t;
  return LBM_OK;
}

int lbm_solver_weighted_momentum(lbm_solver* s, const double* weight, int32_t axis, double* out) {
  clear_error();
  if (!s || !weight || !out) return fail(LBM_EINVAL, "null pointer");
  if (axis < 0 || axis > 2) return fail(LBM_EINVAL, "axis must be 0, 1 or 2");
  const int32_t N = (int32_t)s->p.n_fluid;
  unsigned parts = 0;
  if (N > 0) {
    parts = std::min<unsigned>(grid_for(N), kRedBlocks);
    const int layout = current_layout(s);
    dispatch(s, current_grid(s), [&](auto* F, auto idx) {
      using S = std::remove_pointer_t<decltype(F)>;
      hipLaunchKernelGGL((weighted_momentum<S, decltype(idx)>), dim3(parts), dim3(kBlock), 0, s->stream,
                         (const S*)F, N, idx, layout, s->c, weight, (int)axis, s->ws);
    });
  }
  hipLaunchKernelGGL(finish_totals, dim3(1), dim3(kBlock), 0, s->stream, s->ws, (int)parts, s->ws + 4 * kRedBlocks);
  if (hipMemcpyAsync(out, s->ws + 4 * kRedBlocks, sizeof(double), hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
    return device_status("weighted_momentum (copy)");
  int rc = device_status("weighted_momentum");
  if (rc) return rc;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return device_status("weighted_momentum (sync)");
  return LBM_OK;
}

namespace {
int adjoint_ready(const lbm_solver* s) {
  if (s->p.pattern != LBM_PATTERN_AA || s->p.precision != LBM_F64 || s->trt)
    return fail(LBM_ESTATE, "the adjoint is defined for AA, FP64, BGK");
  return LBM_OK;
}
}  // namespace

int lbm_adjoint_seed_momentum(lbm_solver* s, const double* weight, int32_t axis, int64_t t, double* lam) {
  clear_error();
  if (!s || !weight || !lam) return fail(LBM_EINVAL, "null pointer");
  if (axis < 0 || axis > 2 || t < 0) return fail(LBM_EINVAL, "bad axis or time");
  int rc = adjoint_ready(s);
  if (rc) return rc;
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N == 0) return LBM_OK;
  auto go = [&](auto idx) {
    using I = decltype(idx);
    if (t % 2 == 0)
      hipLaunchKernelGGL((adjoint_seed<I, false>), dim3(grid_for(N)), dim3(kBlock), 0, s->stream, lam, N,
                         idx, weight, (int)axis);
    else
      hipLaunchKernelGGL((adjoint_seed<I, true>), dim3(grid_for(N)), dim3(kBlock), 0, s->stream, lam, N,
                         idx, weight, (int)axis);
  };
  with_index(s, go);
  return device_status("adjoint_seed_momentum");
}

int lbm_solver_step_save(lbm_solver* s, double* save) {
  clear_error();
  if (!s || !save) return fail(LBM_EINVAL, "null pointer");
  int rc = adjoint_ready(s);
  if (rc) return rc;
  if (save == s->b.pdf[0]) return fail(LBM_EINVAL, "save must not be the solver's grid");
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N > 0) launch_step_pbb(s, N, save);
  s->t += 1;
  return device_status("step_save");
}

int lbm_adjoint_step(lbm_solver* s, const double* fwd, int64_t t, double* lam, double* grad) {
  clear_error();
  if (!s || !fwd || !lam) return fail(LBM_EINVAL, "null pointer");
  if (t < 0) return fail(LBM_EINVAL, "t < 0");
  int rc = adjoint_ready(s);
  if (rc) return rc;
  const int32_t N = (int32_t)s->p.n_fluid;
  if (N == 0) return LBM_OK;
  const int chunk = s->remap ? kOddChunk : 0;
  const dim3 grid(chunked_grid(grid_for(N), chunk));
  auto go = [&](auto idx, auto off) {
    using I = decltype(idx);
    using Off = decltype(off);
    if (t % 2 == 0)
      hipLaunchKernelGGL((aa_adjoint<I, false, Off>), grid, dim3(kBlock), 0, s->stream, fwd, lam, N, idx, s->c,
                         s->b.solid_frac, grad, chunk);
    else
      hipLaunchKernelGGL((aa_adjoint<I, true, Off>), grid, dim3(kBlock), 0, s->stream, fwd, lam, N, idx, s->c,
                         s->b.solid_frac, grad, chunk);
  };
  with_index(s, [&](auto idx) { with_slots(s, [&](auto off) { go(idx, off); }); });
  return device_status("adjoint_step");
}

void lbm_solver_free(lbm_solver* s) { delete s; }

int lbm_bench_stream(int32_t kind, const double* src, double* dst, int64_t n, int64_t ld,
                     void* hip_stream) {
  clear_error();
  hipStream_t st = (hipStream_t)hip_stream;
  if (n < 0) return fail(LBM_EINVAL, "n < 0");
  if (n == 0) return LBM_OK;
  switch (kind) {
    case 0:
    case 4: {
      if (!src || !dst) return fail(LBM_EINVAL, "copy needs src and dst");
      if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return fail(LBM_EINVAL, "copy needs 16-byte alignment");
      const int64_t n2 = n / 2;
      if (n2) hipLaunchKernelGGL(bench_copy, dim3(grid_for(n2)), dim3(kBlock), 0, st, (const vec2d*)src,
                                 (vec2d*)dst, n2);
      if (n % 2) hipLaunchKernelGGL(bench_copy_tail, dim3(1), dim3(kBlock), 0, st, src, dst, 2 * n2, n);
      break;
    }
    case 1:
      if (!src || !dst || ld < n) return fail(LBM_EINVAL, "CNT-19A needs src, dst and ld >= n");
      hipLaunchKernelGGL(bench_cnt19, dim3(grid_for(n)), dim3(kBlock), 0, st, src, dst, n, ld);
      break;
    case 2:
      if (!dst || ld < n) return fail(LBM_EINVAL, "U-19A needs dst and ld >= n");
      hipLaunchKernelGGL(bench_u19, dim3(grid_for(n)), dim3(kBlock), 0, st, dst, n, ld, 1.0);
      break;
    case 5:
    case 7:
      if (!dst || ld < (n + kTile - 1) / kTile * kTile) return fail(LBM_EINVAL, "U-19T needs dst and ld >= n rounded to 64");
      if (kind == 5) {
        hipLaunchKernelGGL(bench_u19_tiles, dim3(grid_for(n)), dim3(kBlock), 0, st, dst, n, 1.0, 0);
      } else {  // the FP64 even step's launch
        const unsigned lds = lds_for_device(kEvenWgsPerCu[LBM_F64]);
        hipLaunchKernelGGL(bench_u19_tiles, dim3(chunked_grid(grid_for(n), kEvenChunk)), dim3(kBlock), lds, st, dst,
                           n, 1.0, kEvenChunk);
      }
      break;
    case 6:
    case 8:
      if (!src || !dst || ld < (n + kTile - 1) / kTile * kTile)
        return fail(LBM_EINVAL, "CNT-19T needs src, dst and ld >= n rounded to 64");
      if (kind == 6) {
        hipLaunchKernelGGL(bench_cnt19_tiles, dim3(grid_for(n)), dim3(kBlock), 0, st, src, dst, n, 0);
      } else {  // the streaming launch of the FP64 even step
        const unsigned lds = lds_for_device(kEvenWgsPerCu[LBM_F64]);
        hipLaunchKernelGGL(bench_cnt19_tiles, dim3(chunked_grid(grid_for(n), kEvenChunk)), dim3(kBlock), lds, st,
                           src, dst, n, kEvenChunk);
      }
      break;
    case 3:
      if (!dst) return fail(LBM_EINVAL, "U-1A needs dst");
      hipLaunchKernelGGL(bench_u1, dim3(grid_for(n)), dim3(kBlock), 0, st, dst, n, 1.0);
      break;
    default:
      return fail(LBM_EINVAL, "unknown benchmark kind %d", kind);
  }
  return device_status("bench_stream");
}

}  // extern "C"
