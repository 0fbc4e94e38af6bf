// Differentiation extension: partial bounce-back (PBB) AA steps and their
// hand-written adjoint (FP64, BGK, AA pattern).
//
// PBB gives every fluid node a solid fraction ns in [0, 1] and replaces the
// post-collision PDFs by post_q = (1 - ns) f*_q + ns f_qbar (f* from BGK).
// ns = 0 reproduces the plain step bitwise.
//
// Adjoint of one AA step. A step gathers f_q from slot G_q(n) and scatters
// post_q to slot G_qbar(n): G_q(n) = (q, n) in even steps and L_q(n) in odd
// steps. The adjoint grid Lam uses the same (tile-major) slot layout. Its step gathers
// mu_q = Lam[G_qbar(n)] = dJ/dpost_q and scatters lam_k = dJ/df_k to
// G_k(n). Each node touches the same slot set as in the forward step, so the
// adjoint also runs in place without races, backwards in time.
//
// Transposed Jacobian of post (u = j/rho, feq second order):
//   lam_k = (1 - ns) [(1 - omega) mu_k + omega (A + c_k . B)] + ns mu_kbar,
//   A = sum_q mu_q w_q (1 - 9/2 (c_q.u)^2 + 3/2 u.u),
//   B = sum_q mu_q w_q (3 c_q + 9 (c_q.u) c_q - 3 u),
// and the gradient contribution dJ/dns(n) += sum_q mu_q (f_qbar - f*_q).
#pragma once

#include "kernels.hpp"

namespace lbm {

template <class Idx, bool ODD, class Off>
__device__ __forceinline__ void step_slots(int32_t n, const Idx& idx, Off (&g)[Q]) {
  if constexpr (ODD) {
    int32_t a[18];
    idx.get(n, a);
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = aa_slot<Off>(q, n, a);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = pdf_slot<Off>(q, n);
  }
}

// One AA step with partial bounce-back (ns = NULL: every ns is 0). SAVE
// also writes the PDFs f(t) it reads into `save`, in the grid's slots of
// time t: the forward state the adjoint of this step reads. Off is the slot
// type (kernels.hpp).
template <class Idx, bool ODD, bool SAVE, class Off>
__global__ void __launch_bounds__(kBlock)
aa_step_pbb(double* __restrict__ F, int32_t N, Idx idx, Collision c,
            const double* __restrict__ ns, double* __restrict__ save, int chunk) {
  const int64_t n64 = tile_index(chunk) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  Off g[Q];
  step_slots<Idx, ODD>(n, idx, g);
  double f[Q], fs[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = fs[q] = F[g[q]];
  if constexpr (SAVE) {
#pragma unroll
    for (int q = 0; q < Q; ++q) save[g[q]] = f[q];
  }
  collide_f64(fs, c);
  const double s = ns ? ns[n] : 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) F[g[kOpp[q]]] = ((1.0 - s) * fs[q]) + (s * f[kOpp[q]]);
}

template <class Idx, bool ODD, class Off>
__global__ void __launch_bounds__(kBlock)
aa_adjoint(const double* __restrict__ F, double* __restrict__ Lam, int32_t N, Idx idx,
           Collision c, const double* __restrict__ ns, double* __restrict__ grad, int chunk) {
  const int64_t n64 = tile_index(chunk) * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  Off g[Q];
  step_slots<Idx, ODD>(n, idx, g);
  double f[Q], mu[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = F[g[q]];
#pragma unroll
  for (int q = 0; q < Q; ++q) mu[q] = Lam[g[kOpp[q]]];
  const double rho = density(f);
  const double ux = momentum<0>(f) / rho, uy = momentum<1>(f) / rho, uz = momentum<2>(f) / rho;
  const double usq = (ux * ux + uy * uy) + uz * uz;
  double A = 0.0, Bx = 0.0, By = 0.0, Bz = 0.0, dg = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cu = cdot<double>(q, ux, uy, uz);
    const double feq = (kW[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq);
    const double fstar = (f[q] - c.omega * (f[q] - feq)) + c.S[q];
    dg += mu[q] * (f[kOpp[q]] - fstar);
    const double wm = kW[q] * mu[q];
    A += wm * (1.0 - 4.5 * cu * cu + 1.5 * usq);
    const double k = 3.0 + 9.0 * cu;
    Bx += wm * (k * kC[q][0] - 3.0 * ux);
    By += wm * (k * kC[q][1] - 3.0 * uy);
    Bz += wm * (k * kC[q][2] - 3.0 * uz);
  }
  const double s = ns ? ns[n] : 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cB = cdot<double>(q, Bx, By, Bz);
    const double lam = (1.0 - s) * ((1.0 - c.omega) * mu[q] + c.omega * (A + cB)) + s * mu[kOpp[q]];
    Lam[g[q]] = lam;
  }
  if (grad) grad[n] += dg;
}

// Lam = dJ/df(t) for J = sum_n w_n j_axis(n, t), in the slot layout of time t.
template <class Idx, bool ODD>
__global__ void __launch_bounds__(kBlock)
adjoint_seed(double* __restrict__ Lam, int32_t N, Idx idx, const double* __restrict__ w,
             int axis) {
  const int64_t n64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (n64 >= N) return;
  const int32_t n = (int32_t)n64;
  int64_t g[Q];
  step_slots<Idx, ODD>(n, idx, g);
  const double wn = w[n];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int cq = axis == 0 ? kC[q][0] : (axis == 1 ? kC[q][1] : kC[q][2]);
    Lam[g[q]] = wn * (double)cq;
  }
}

}  // namespace lbm
