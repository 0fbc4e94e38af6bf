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
  double omega;      // 1 / tau (BGK rate; TRT rate of the symmetric part)
  double omega_m;    // TRT rate of the antisymmetric part
  double S[Q];       // 3 w_q (c_q . F)
  double rho0;       // reference density of deviation storage
  float omega_f;
  float omega_m_f;
  float S_f[Q];
  float rho0_f;
  float h_scale[Q];    // FP16 storage: stored value = deviation * h_scale[q]
  float h_unscale[Q];  // 1 / h_scale[q] (exact: powers of two times 1/3, 1/18, 1/36)
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

// TRT collision (Sect. 2), FP64, in place. With f+- = (f_q +- f_qbar) / 2
// and the symmetric / antisymmetric equilibrium parts
// e+ = (w_q rho)((1 + (9/2 cu) cu) - 3/2 u.u), e- = (w_q rho)(3 cu):
// f*_q = ((f_q - omega (f+ - e+)) - omega_m (f- - e-)) + S_q.
// Opposite directions are updated as pairs, so no copy of f is kept.
__device__ __forceinline__ void collide_trt_f64(double (&f)[Q], const Collision& c) {
  const double rho = density(f);
  const double jx = momentum<0>(f);
  const double jy = momentum<1>(f);
  const double jz = momentum<2>(f);
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const double usq = (ux * ux + uy * uy) + uz * uz;
  {
    const double wr = kW[0] * rho;
    const double ep = wr * ((1.0 + (4.5 * 0.0) * 0.0) - 1.5 * usq);
    const double em = wr * (3.0 * 0.0);
    const double fp = (f[0] + f[0]) * 0.5, fm = (f[0] - f[0]) * 0.5;
    f[0] = ((f[0] - c.omega * (fp - ep)) - c.omega_m * (fm - em)) + c.S[0];
  }
#pragma unroll
  for (int q = 1; q < Q; q += 2) {
    const int b = q + 1;  // kOpp[q]
    const double cu = cdot<double>(q, ux, uy, uz);
    const double cub = cdot<double>(b, ux, uy, uz);
    const double wr = kW[q] * rho;
    const double ep = wr * ((1.0 + (4.5 * cu) * cu) - 1.5 * usq);
    const double em = wr * (3.0 * cu);
    const double epb = wr * ((1.0 + (4.5 * cub) * cub) - 1.5 * usq);
    const double emb = wr * (3.0 * cub);
    const double fp = (f[q] + f[b]) * 0.5, fm = (f[q] - f[b]) * 0.5;
    const double fpb = (f[b] + f[q]) * 0.5, fmb = (f[b] - f[q]) * 0.5;
    const double nq = ((f[q] - c.omega * (fp - ep)) - c.omega_m * (fm - em)) + c.S[q];
    const double nb = ((f[b] - c.omega * (fpb - epb)) - c.omega_m * (fmb - emb)) + c.S[b];
    f[q] = nq;
    f[b] = nb;
  }
}

// ------------------------------------------------------------------------
// Deviation storage: the grid holds d_q = f_q - w_q rho0 (FP32, or FP16
// scaled by 2^s / w_q), arithmetic in FP32. Since sum_q w_q = 1 and
// sum_q w_q c_q = 0, rho = rho0 + sum_q d_q and j = sum_q c_q d_q, and the
// equilibrium deviation is w_q (drho + rho (3 cu + 9/2 cu^2 - 3/2 u.u)), so
// the O(1) rest part never enters a rounding step.

constexpr float kWf[Q] = {1.0f / 3.0f,  1.0f / 18.0f, 1.0f / 18.0f, 1.0f / 18.0f, 1.0f / 18.0f,
                          1.0f / 18.0f, 1.0f / 18.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f,
                          1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f,
                          1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f};

__device__ __forceinline__ void collide_dev_f32(float (&d)[Q], const Collision& c) {
#pragma clang fp contract(fast)
  const float drho = density(d);
  const float rho = c.rho0_f + drho;
  const float jx = momentum<0>(d);
  const float jy = momentum<1>(d);
  const float jz = momentum<2>(d);
  const float ir = 1.0f / rho;
  const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const float cu = cdot<float>(q, ux, uy, uz);
    const float deq = kWf[q] * (drho + rho * (cu * (3.0f + 4.5f * cu) - usq15));
    d[q] = d[q] - c.omega_f * (d[q] - deq) + c.S_f[q];
  }
}

// TRT on deviations: the rest part w_q rho0 is symmetric, so d- = f- and
// d+ = f+ - w_q rho0; the equilibrium parts become
// e+ - w_q rho0 = w_q (drho + rho (9/2 cu^2 - 3/2 u.u)) and e- = w_q rho 3 cu.
__device__ __forceinline__ void collide_trt_dev_f32(float (&d)[Q], const Collision& c) {
#pragma clang fp contract(fast)
  const float drho = density(d);
  const float rho = c.rho0_f + drho;
  const float jx = momentum<0>(d);
  const float jy = momentum<1>(d);
  const float jz = momentum<2>(d);
  const float ir = 1.0f / rho;
  const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  d[0] = d[0] - c.omega_f * (d[0] - kWf[0] * (drho - rho * usq15)) + c.S_f[0];
#pragma unroll
  for (int q = 1; q < Q; q += 2) {
    const int b = q + 1;
    const float cu = cdot<float>(q, ux, uy, uz);  // cu of b is -cu
    const float epd = kWf[q] * (drho + rho * (4.5f * cu * cu - usq15));
    const float em = kWf[q] * rho * 3.0f * cu;
    const float dp = 0.5f * (d[q] + d[b]), dm = 0.5f * (d[q] - d[b]);
    const float sym = c.omega_f * (dp - epd), anti = c.omega_m_f * (dm - em);
    const float nq = d[q] - sym - anti + c.S_f[q];
    const float nb = d[b] - sym + anti + c.S_f[b];
    d[q] = nq;
    d[b] = nb;
  }
}

// Deviation of the equilibrium in FP64 (initialisation of deviation storage).
__device__ __forceinline__ double equilibrium_dev_f64(int q, double rho, double rho0, double ux,
                                                      double uy, double uz) {
  const double usq = (ux * ux + uy * uy) + uz * uz;
  const double cu = cdot<double>(q, ux, uy, uz);
  return kW[q] * ((rho - rho0) + rho * ((3.0 * cu + (4.5 * cu) * cu) - 1.5 * usq));
}

// Storage traits. value64: the stored quantity in FP64 (f_q for FP64
// storage, the deviation d_q otherwise); from64: its rounding to storage.
template <class S>
struct Prec;

template <>
struct Prec<double> {
  static constexpr bool kDeviation = false;
  template <bool TRT>
  __device__ static void collide(double (&v)[Q], const Collision& c) {
    if constexpr (TRT)
      collide_trt_f64(v, c);
    else
      collide_f64(v, c);
  }
  __device__ static double value64(int, double v, const Collision&) { return v; }
  __device__ static double from64(int, double x, const Collision&) { return x; }
};

template <>
struct Prec<float> {
  static constexpr bool kDeviation = true;
  template <bool TRT>
  __device__ static void collide(float (&v)[Q], const Collision& c) {
    if constexpr (TRT)
      collide_trt_dev_f32(v, c);
    else
      collide_dev_f32(v, c);
  }
  __device__ static double value64(int, float v, const Collision&) { return (double)v; }
  __device__ static float from64(int, double d, const Collision&) { return (float)d; }
};

// double -> binary16 with a single rounding to nearest-even. A plain
// double -> float -> half chain rounds twice and can land on the wrong side
// of a half-way point. Here the first rounding, to float, is made
// round-to-odd (truncate, then set the last bit if anything was cut off):
// float keeps 13 more significand bits than half, so rounding that result to
// nearest gives the correctly rounded half of x (Boldo and Melquiond,
// "Emulation of FMA and correctly rounded sums: proved algorithms using
// rounding to odd", IEEE Trans. Computers 57(4), 2008).
__device__ __forceinline__ _Float16 half_from_double(double x) {
  float f = (float)x;
  if ((double)f != x && f == f) {  // inexact (x is not NaN)
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(x)) b -= 1;  // one step towards zero
    f = __uint_as_float(b | 1u);
  }
  return (_Float16)f;
}

template <>
struct Prec<_Float16> {
  static constexpr bool kDeviation = true;
  template <bool TRT>
  __device__ static void collide(_Float16 (&v)[Q], const Collision& c) {
    float d[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) d[q] = (float)v[q] * c.h_unscale[q];
    if constexpr (TRT)
      collide_trt_dev_f32(d, c);
    else
      collide_dev_f32(d, c);
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = (_Float16)(d[q] * c.h_scale[q]);
  }
  __device__ static double value64(int q, _Float16 v, const Collision& c) {
    return (double)v * (double)c.h_unscale[q];
  }
  __device__ static _Float16 from64(int q, double d, const Collision& c) {
    return half_from_double(d * (double)c.h_scale[q]);
  }
};

}  // namespace lbm
