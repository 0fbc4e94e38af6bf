// D3Q19 constants and the BGK collision for the GPU kernels.
//
// Sect. 2: a D3Q19 node holds 19 PDFs f_q; one time step of the lattice
// Boltzmann equation, eq. (1), collides them and propagates the
// post-collision values to the neighbours. The paper uses double precision
// (Sect. 4) and names a TRT collision without formulas; this library uses BGK
// with a second-order equilibrium (c_s^2 = 1/3), a constant body-force
// density F added as S_q = 3 w_q (c_q . F), and u = j / rho.
//
// The FP64 collision evaluates every sum and product in one fixed order (left
// folds in ascending q, axis order x, y, z, zero-coefficient terms skipped),
// and the library is compiled without floating-point contraction, so every
// site gets one well-defined IEEE result regardless of propagation pattern,
// addressing mode or node order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

constexpr int Q = 19;

// velocity set c_q
constexpr int kC[Q][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

// opposite direction: c_opp(q) = -c_q
constexpr int kOpp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

// lattice weights (each one IEEE division, folded at compile time)
constexpr double kW[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                          1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Per-launch collision constants (host-computed, passed by value).
struct Collision {
  double omega;     // 1 / tau
  double S[Q];      // 3 w_q (c_q . F)
  float omega_f;
  float S_f[Q];
  float rho0_f;     // reference density of deviation storage
  float pad_;
};

// c_q . v folded over the nonzero components of c_q in axis order.
template <class T>
__host__ __device__ __forceinline__ T cdot(int q, T vx, T vy, T vz) {
  const T v[3] = {vx, vy, vz};
  T acc = T(0);
  bool first = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (kC[q][a] != 0) {
      const T t = kC[q][a] > 0 ? v[a] : -v[a];
      acc = first ? t : acc + t;
      first = false;
    }
  }
  return acc;
}

// j_a = sum_q c_qa f_q, left fold in ascending q over c_qa != 0.
template <int A, class T>
__device__ __forceinline__ T momentum(const T (&f)[Q]) {
  T acc = T(0);
  bool first = true;
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    if (kC[q][A] != 0) {
      const T t = kC[q][A] > 0 ? f[q] : -f[q];
      acc = first ? t : acc + t;
      first = false;
    }
  }
  return acc;
}

template <class T>
__device__ __forceinline__ T density(const T (&f)[Q]) {
  T rho = f[0];
#pragma unroll
  for (int q = 1; q < Q; ++q) rho = rho + f[q];
  return rho;
}

// Equilibrium feq_q(rho, u) = (w_q rho) (((1 + 3 cu) + (9/2 cu) cu) - 3/2 u.u).
__device__ __forceinline__ void equilibrium_f64(double rho, double ux, double uy, double uz,
                                                double (&feq)[Q]) {
  const double usq = (ux * ux + uy * uy) + uz * uz;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cu = cdot<double>(q, ux, uy, uz);
    feq[q] = (kW[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq);
  }
}

// BGK collision with body force, FP64, in place:
// f*_q = (f_q - omega (f_q - feq_q)) + S_q.
__device__ __forceinline__ void collide_f64(double (&f)[Q], const Collision& c) {
  const double rho = density(f);
  const double jx = momentum<0>(f);
  const double jy = momentum<1>(f);
  const double jz = momentum<2>(f);
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const double usq = (ux * ux + uy * uy) + uz * uz;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cu = cdot<double>(q, ux, uy, uz);
    const double feq = (kW[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq);
    f[q] = (f[q] - c.omega * (f[q] - feq)) + c.S[q];
  }
}

}  // namespace lbm
