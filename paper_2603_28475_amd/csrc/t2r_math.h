// Device math of the PNCG-IPC step energy: neo-Hookean tet terms, IPC barrier,
// primitive distances with their derivatives, and the friction mollifier.
// Everything here is FP64 unless a function name ends in 32.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace t2r {

// ---------------------------------------------------------------------------
// Neo-Hookean tet (reading of the hyperelastic potential, Supp. A eq. varopt):
//   psi(F) = mu/2 (|F|^2 - 3) - mu ln J + lam/2 (ln J)^2,   F = Ds Dm^-1.
// With g_i the rows of Dm^-1 (g_0 = -(g_1+g_2+g_3)):
//   grad_i      = V P(F) g_i,  P = mu (F - F^-T) + lam ln J F^-T
//   diag_(i,a)  = V [mu |g_i|^2 + (mu + lam (1 - ln J)) ((F^-T g_i)_a)^2]
//   p^T H_e p   = V [mu |dF|^2 + (mu - lam ln J) tr((F^-1 dF)^2) + lam (tr F^-1 dF)^2]
// ---------------------------------------------------------------------------

// Gradient and diagonal of one tet from its deformation gradient F (with
// ln J given), handed to emit(i, a, grad, diag) per (vertex i, axis a) as soon
// as each is known, so no per-tet array of 24 results stays live. F is
// overwritten.
template <typename T, typename Emit>
__device__ __forceinline__ void tet_grad_diag_from_F(T F[9], const T Dm[9], T V, T mu, T lam, T lnJ,
                                                     Emit&& emit) {
  T C[9];  // cofactor matrix, J F^-T
  C[0] = F[4] * F[8] - F[5] * F[7];
  C[1] = F[5] * F[6] - F[3] * F[8];
  C[2] = F[3] * F[7] - F[4] * F[6];
  C[3] = F[2] * F[7] - F[1] * F[8];
  C[4] = F[0] * F[8] - F[2] * F[6];
  C[5] = F[1] * F[6] - F[0] * F[7];
  C[6] = F[1] * F[5] - F[2] * F[4];
  C[7] = F[2] * F[3] - F[0] * F[5];
  C[8] = F[0] * F[4] - F[1] * F[3];
  const T invJ = T(1) / (F[0] * C[0] + F[1] * C[1] + F[2] * C[2]);
  // reuse F for V P and C for F^-T
  const T cP = lam * lnJ - mu;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    C[k] *= invJ;
    F[k] = V * (mu * F[k] + cP * C[k]);
  }
  const T cd = V * (mu + lam * (T(1) - lnJ));
  const T Vmu = V * mu;
  T gs0 = T(0), gs1 = T(0), gs2 = T(0);
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    const T gi0 = Dm[(i - 1) * 3 + 0], gi1 = Dm[(i - 1) * 3 + 1], gi2 = Dm[(i - 1) * 3 + 2];
    const T gg = Vmu * (gi0 * gi0 + gi1 * gi1 + gi2 * gi2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T ga = F[a * 3 + 0] * gi0 + F[a * 3 + 1] * gi1 + F[a * 3 + 2] * gi2;
      const T w = C[a * 3 + 0] * gi0 + C[a * 3 + 1] * gi1 + C[a * 3 + 2] * gi2;
      emit(i, a, ga, gg + cd * w * w);
      if (a == 0) gs0 += ga; else if (a == 1) gs1 += ga; else gs2 += ga;
    }
  }
  {
    const T g00 = -(Dm[0] + Dm[3] + Dm[6]), g01 = -(Dm[1] + Dm[4] + Dm[7]),
            g02 = -(Dm[2] + Dm[5] + Dm[8]);
    const T gg = Vmu * (g00 * g00 + g01 * g01 + g02 * g02);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T w = C[a * 3 + 0] * g00 + C[a * 3 + 1] * g01 + C[a * 3 + 2] * g02;
      emit(0, a, -(a == 0 ? gs0 : (a == 1 ? gs1 : gs2)), gg + cd * w * w);
    }
  }
}

// FP64 deformation gradient F = Ds Dm, J = det F and ln J; false for J <= 0.
// Returns the FP64 energy V psi(F) in `energy`.
template <typename TD>
__device__ __forceinline__ bool tet_F_energy(const double Ds[9], const TD Dm[9], double V, double mu,
                                             double lam, double F[9], double& lnJ, double& energy) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      F[a * 3 + b] = Ds[a * 3 + 0] * (double)Dm[0 * 3 + b] + Ds[a * 3 + 1] * (double)Dm[1 * 3 + b] +
                     Ds[a * 3 + 2] * (double)Dm[2 * 3 + b];
  const double J = F[0] * (F[4] * F[8] - F[5] * F[7]) + F[1] * (F[5] * F[6] - F[3] * F[8]) +
                   F[2] * (F[3] * F[7] - F[4] * F[6]);
  if (!(J > 0.0)) return false;
  lnJ = log(J);
  double I1 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) I1 += F[k] * F[k];
  energy = V * (0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
  return true;
}

// FP64 tet: energy, gradient and diagonal all in double.
template <typename Emit>
__device__ __forceinline__ bool tet_grad_diag64(const double Ds[9], const double Dm[9], double V, double mu,
                                                double lam, double& energy, Emit&& emit) {
  double F[9], lnJ;
  if (!tet_F_energy(Ds, Dm, V, mu, lam, F, lnJ, energy)) return false;
  tet_grad_diag_from_F<double>(F, Dm, V, mu, lam, lnJ, emit);
  return true;
}

// Below this volume ratio J the mixed path computes a tet's element terms in
// FP64. FP32 element terms lose about cond(F) x 2^-24 in relative accuracy, and
// a tet squashed towards zero volume has cond(F) ~ 1/J: near J = 1e-7 the FP32
// cofactors no longer carry the sign of det F, the stress points the wrong way
// and the search direction stops being a descent direction for the FP64 energy
// (a collapsed surface tet under a flat indenter stalled a solve that way). At
// J >= 0.1 the FP32 terms stay within about 1e-6 relative.
constexpr double kMixedMinJ = 0.1;

// Mixed tet: F, J, ln J and the energy in double (the line search compares
// energies), gradient and diagonal in float from the rounded F, or in double
// when J < kMixedMinJ. emit receives float or double values.
template <typename Emit>
__device__ __forceinline__ bool tet_grad_diag_mixed(const double Ds[9], const float Dm[9], float V, double mu,
                                                    double lam, double& energy, Emit&& emit) {
  double F[9], lnJ;
  if (!tet_F_energy(Ds, Dm, (double)V, mu, lam, F, lnJ, energy)) return false;
  if (lnJ < log(kMixedMinJ)) {
    double Dm64[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Dm64[k] = (double)Dm[k];
    tet_grad_diag_from_F<double>(F, Dm64, (double)V, mu, lam, lnJ, emit);
    return true;
  }
  float F32[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) F32[k] = (float)F[k];
  tet_grad_diag_from_F<float>(F32, Dm, V, (float)mu, (float)lam, (float)lnJ, emit);
  return true;
}

template <typename T>
__device__ __forceinline__ T tet_curvature(const T Ds[9], const T dDs[9], const T Dm[9], T V, T mu, T lam) {
  T F[9], dF[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      F[a * 3 + b] = Ds[a * 3 + 0] * Dm[0 * 3 + b] + Ds[a * 3 + 1] * Dm[1 * 3 + b] +
                     Ds[a * 3 + 2] * Dm[2 * 3 + b];
      dF[a * 3 + b] = dDs[a * 3 + 0] * Dm[0 * 3 + b] + dDs[a * 3 + 1] * Dm[1 * 3 + b] +
                      dDs[a * 3 + 2] * Dm[2 * 3 + b];
    }
  T C[9];
  C[0] = F[4] * F[8] - F[5] * F[7];
  C[1] = F[5] * F[6] - F[3] * F[8];
  C[2] = F[3] * F[7] - F[4] * F[6];
  C[3] = F[2] * F[7] - F[1] * F[8];
  C[4] = F[0] * F[8] - F[2] * F[6];
  C[5] = F[1] * F[6] - F[0] * F[7];
  C[6] = F[1] * F[5] - F[2] * F[4];
  C[7] = F[2] * F[3] - F[0] * F[5];
  C[8] = F[0] * F[4] - F[1] * F[3];
  const T J = F[0] * C[0] + F[1] * C[1] + F[2] * C[2];
  if (!(J > T(0))) return T(0);
  const T invJ = T(1) / J;
  const T lnJ = log(J);
  // F^-1 = C^T / J ;  A = F^-1 dF
  T A[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      A[a * 3 + b] = (C[0 * 3 + a] * dF[0 * 3 + b] + C[1 * 3 + a] * dF[1 * 3 + b] +
                      C[2 * 3 + a] * dF[2 * 3 + b]) * invJ;
  const T trA = A[0] + A[4] + A[8];
  T trAA = T(0), dd = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) trAA += A[a * 3 + b] * A[b * 3 + a];
#pragma unroll
  for (int k = 0; k < 9; ++k) dd += dF[k] * dF[k];
  return V * (mu * dd + (mu - lam * lnJ) * trAA + lam * trA * trA);
}

// ---------------------------------------------------------------------------
// IPC log barrier on the unsquared distance (Supp. A, eq. ipc_energy):
//   b(d) = -(d - dh)^2 ln(d / dh) on (0, dh), 0 beyond.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void barrier3(double d, double dh, double& b, double& b1, double& b2) {
  const double e = d - dh;
  const double l = log(d / dh);
  b = -e * e * l;
  b1 = -2.0 * e * l - e * e / d;
  b2 = -2.0 * l - 4.0 * e / d + (e * e) / (d * d);
}

// Edge-edge mollifier (option; IPC, whose contact model Supp. A follows): the
// barrier of a gel-edge / indenter-edge pair is weighted by m(c), c = |a x b|^2
// of the two edge vectors, m(c) = (c/e)(2 - c/e) below e and 1 above, with
// e = kEdgeMollRel |a_rest|^2 |b_rest|^2; m, m' and m'' at c < e.
constexpr double kEdgeMollRel = 1e-3;
__device__ __forceinline__ void edge_mollifier3(double c, double e, double& m, double& m1, double& m2) {
  const double ie = 1.0 / e, s = c * ie;
  m = s * (2.0 - s);
  m1 = 2.0 * ie * (1.0 - s);
  m2 = -2.0 * ie * ie;
}

// Friction mollifier (Supp. A, eq. friction_mollifier) pieces at s >= 0:
//   f(s), f'(s)/s, and (f''(s) - f'(s)/s)/s^2 * s^2 / s  written as `corr` so that
//   Hess_Delta = mulam [ fos T + corr uhat uhat^T ] with uhat = T Delta / s.
__device__ __forceinline__ void mollifier3(double s, double eps, double& f, double& fos, double& corr) {
  if (s < eps) {
    f = -s * s * s / (3.0 * eps * eps) + s * s / eps + eps / 3.0;
    fos = -s / (eps * eps) + 2.0 / eps;
    corr = -s / (eps * eps);
  } else {
    f = s;
    fos = 1.0 / s;
    corr = -1.0 / s;
  }
}

// ---------------------------------------------------------------------------
// Closest features between closed primitives.
// A pair is described over four points z0..z3 by coefficients c (the vector
// between the closest points is r = sum c_i z_i, d = |r|) and, for the k free
// barycentric parameters w of the active feature, Cw = dc/dw. Derivatives then
// follow from the value function d^2 = min_w |sum c_i(w) z_i|^2 (envelope and
// implicit-function theorems):
//   grad_{z_i} d = c_i r / d
//   Hess(d)_(i a)(i a) = (c_i^2 - u^T M^-1 u)/d - (c_i n_a)^2/d,
//        u_w = Cw_iw r_a + c_i D_w,a,  D_w = sum_i Cw_iw z_i,  M = D D^T
//   p^T Hess(d) p = (|q|^2 - v^T M^-1 v)/d - (n.q)^2/d,
//        q = sum c_i p_i,  v_w = sum_i Cw_iw (r.p_i) + c_i (D_w.p_i)
// ---------------------------------------------------------------------------
// Cw has entries in {-1, 0, 1}: two bits per (point i, free parameter w) at
// bit 4 i + 2 w (0: 0, 1: +1, 3: -1), which keeps a feature in few registers.
struct Feature {
  double c[4];
  int cw;
  int k;
};

__host__ __device__ constexpr int cw_bits(int i, int w, int sign) { return (sign > 0 ? 1 : 3) << (4 * i + 2 * w); }

__device__ __forceinline__ double cw_of(const Feature& f, int i, int w) {
  const int b = (f.cw >> (4 * i + 2 * w)) & 3;
  return b == 0 ? 0.0 : (b == 1 ? 1.0 : -1.0);
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Point p against triangle (a, b, c) by Voronoi-region tests of the closest
// point (Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5).
// Point order: z0 = p, z1 = a, z2 = b, z3 = c; r = p - closest.
__device__ __forceinline__ void classify_pt(const double p[3], const double a[3], const double b[3],
                                   const double c[3], Feature& f) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i];
    ac[i] = c[i] - a[i];
    ap[i] = p[i] - a[i];
    bp[i] = p[i] - b[i];
    cp[i] = p[i] - c[i];
  }
  f.cw = 0;
  f.c[0] = 1.0;
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) {  // vertex a
    f.c[1] = -1.0; f.c[2] = 0.0; f.c[3] = 0.0; f.k = 0;
    return;
  }
  const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) {  // vertex b
    f.c[1] = 0.0; f.c[2] = -1.0; f.c[3] = 0.0; f.k = 0;
    return;
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {  // edge ab
    const double v = d1 / (d1 - d3);
    f.c[1] = -(1.0 - v); f.c[2] = -v; f.c[3] = 0.0; f.k = 1;
    f.cw = cw_bits(1, 0, 1) | cw_bits(2, 0, -1);
    return;
  }
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) {  // vertex c
    f.c[1] = 0.0; f.c[2] = 0.0; f.c[3] = -1.0; f.k = 0;
    return;
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {  // edge ac
    const double w = d2 / (d2 - d6);
    f.c[1] = -(1.0 - w); f.c[2] = 0.0; f.c[3] = -w; f.k = 1;
    f.cw = cw_bits(1, 0, 1) | cw_bits(3, 0, -1);
    return;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {  // edge bc
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    f.c[1] = 0.0; f.c[2] = -(1.0 - w); f.c[3] = -w; f.k = 1;
    f.cw = cw_bits(2, 0, 1) | cw_bits(3, 0, -1);
    return;
  }
  const double den = 1.0 / (va + vb + vc);  // face interior
  const double v = vb * den, w = vc * den;
  f.c[1] = -(1.0 - v - w); f.c[2] = -v; f.c[3] = -w; f.k = 2;
  f.cw = cw_bits(1, 0, 1) | cw_bits(2, 0, -1) | cw_bits(1, 1, 1) | cw_bits(3, 1, -1);
}

// Edge-edge below this relative sin^2 of the angle is treated as parallel.
constexpr double kParallelSin2 = 1e-14;

// Segments [a0,a1] and [b0,b1]: clamped closest points (Ericson 2005, Sec. 5.1.9).
// Point order: z0 = a0, z1 = a1, z2 = b0, z3 = b1; r = (a0 + s e_a) - (b0 + t e_b).
__device__ __forceinline__ void classify_ee(const double a0[3], const double a1[3], const double b0[3],
                                   const double b1[3], Feature& f) {
  double d1[3], d2[3], r[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    d1[i] = a1[i] - a0[i];
    d2[i] = b1[i] - b0[i];
    r[i] = a0[i] - b0[i];
  }
  const double A = dot3(d1, d1), E = dot3(d2, d2), F = dot3(d2, r);
  const double C = dot3(d1, r), B = dot3(d1, d2);
  const double den = A * E - B * B;
  double s = 0.0, t;
  if (den > kParallelSin2 * A * E) {
    s = (B * F - C * E) / den;
    s = fmin(fmax(s, 0.0), 1.0);
  }
  t = (B * s + F) / E;
  if (t < 0.0) {
    t = 0.0;
    s = fmin(fmax(-C / A, 0.0), 1.0);
  } else if (t > 1.0) {
    t = 1.0;
    s = fmin(fmax((B - C) / A, 0.0), 1.0);
  }
  f.c[0] = 1.0 - s; f.c[1] = s; f.c[2] = -(1.0 - t); f.c[3] = -t;
  f.cw = 0;
  const bool si = (s > 0.0) && (s < 1.0);
  const bool ti = (t > 0.0) && (t < 1.0);
  // free parameters in order (s first): constant indices only, no dynamic indexing
  if (si) f.cw |= cw_bits(0, 0, -1) | cw_bits(1, 0, 1);
  if (ti) {
    if (si) f.cw |= cw_bits(2, 1, 1) | cw_bits(3, 1, -1);
    else f.cw |= cw_bits(2, 0, 1) | cw_bits(3, 0, -1);
  }
  f.k = (si ? 1 : 0) + (ti ? 1 : 0);
}

// Inverse of the k x k Gram matrix M (k <= 2); returns false if singular.
__device__ __forceinline__ bool gram_inverse(const double D[2][3], int k, double Mi[2][2]) {
  Mi[0][0] = Mi[0][1] = Mi[1][0] = Mi[1][1] = 0.0;
  if (k == 0) return true;
  const double m00 = dot3(D[0], D[0]);
  if (k == 1) {
    if (!(m00 > 0.0)) return false;
    Mi[0][0] = 1.0 / m00;
    return true;
  }
  const double m01 = dot3(D[0], D[1]), m11 = dot3(D[1], D[1]);
  const double det = m00 * m11 - m01 * m01;
  if (!(det > 0.0)) return false;
  const double id = 1.0 / det;
  Mi[0][0] = m11 * id;
  Mi[1][1] = m00 * id;
  Mi[0][1] = Mi[1][0] = -m01 * id;
  return true;
}

}  // namespace t2r
