// Per-site device mathematics of the relativistic lattice Boltzmann step
// (arXiv:1703.04605): Bessel ratio, equation of state inversion, Landau frame,
// projection coefficients.  All in float64.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/rlbm.h"
#include "bessel_ratio_coeffs.h"
#include "rlbm_tables.h"

namespace rlbm {

// R(z) = K_1(z)/K_2(z), the Bessel ratio of the equation of state
// (eq. relativistic-eos).  For z < 1.5: the ascending series of K_0 and K_1
// (integer-order expansions with the logarithmic term, e.g. Abramowitz &
// Stegun 9.6.11/9.6.13) and K_2 = K_0 + 2 K_1/z; otherwise a Chebyshev
// expansion in t = 3/z - 1 (coefficients generated from mpmath).
__device__ __forceinline__ double k1k2_ratio(double z) {
  if (z < RLBM_BESSEL_Z_SPLIT) {
    const double euler_gamma = 0.57721566490153286061;
    const double y = 0.25 * z * z;
    double t0 = 1.0, t1 = 1.0;     // y^k/(k!)^2, y^k/(k!(k+1)!)
    double I0 = 1.0, I1s = 1.0;    // I0(z), 2 I1(z)/z
    double S0 = 0.0;               // sum H_k y^k/(k!)^2
    double S1 = 1.0 - 2.0 * euler_gamma;  // sum (2H_k + 1/(k+1) - 2 gamma) y^k/(k!(k+1)!)
    double H = 0.0;
#pragma unroll
    for (int k = 1; k < 13; ++k) {
      const double kk = (double)k;
      H += 1.0 / kk;
      t0 *= y / (kk * kk);
      t1 *= y / (kk * (kk + 1.0));
      I0 += t0;
      I1s += t1;
      S0 = fma(H, t0, S0);
      S1 = fma(2.0 * H + 1.0 / (kk + 1.0) - 2.0 * euler_gamma, t1, S1);
    }
    const double L = log(0.5 * z);
    const double K0 = S0 - (L + euler_gamma) * I0;
    const double K1 = 1.0 / z + 0.5 * z * (L * I1s - 0.5 * S1);
    return K1 / (K0 + 2.0 * K1 / z);
  }
  const double t = 2.0 * RLBM_BESSEL_Z_SPLIT / z - 1.0;
  const double t2 = 2.0 * t;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int j = RLBM_BESSEL_NCHEB - 1; j >= 1; --j) {
    const double b0 = fma(t2, b1, rlbm_bessel_ratio_cheb[j] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(t, b1, rlbm_bessel_ratio_cheb[0] - b2);
}

// Inverts e = eps/n = 3T + zeta R(zeta/T) (eq. relativistic-eos, T_R = 1)
// by Newton's method on T.  The heat capacity per particle d e/dT lies in
// [3/2, 3] and increases with T, so e(T) is convex and Newton iterates started
// above the root, at min((e - zeta)/1.5, e/3), decrease monotonically to it.
// d e/dT = 3 - z^2 R^2 - 3 z R + z^2 follows from R' = R^2 + 3R/z - 1.
__device__ __forceinline__ double eos_temperature(double e, double zeta, unsigned& flags) {
  double t = fmin((e - zeta) * (1.0 / 1.5), e * (1.0 / 3.0));
  if (!(t > 0.0)) {
    flags |= RLBM_H_RANGE;
    return t;
  }
  bool done = false;
  for (int it = 0; it < 40; ++it) {
    const double z = zeta / t;
    const double r = k1k2_ratio(z);
    const double F = fma(3.0, t, fma(zeta, r, -e));
    const double zr = z * r;
    const double dF = 3.0 - zr * zr - 3.0 * zr + z * z;
    const double d = F / dF;
    t -= d;
    if (done) break;
    if (fabs(d) <= 1e-9 * t) done = true;  // quadratic convergence: one more step
  }
  if (!done) flags |= RLBM_H_EOS;
  return t;
}

// Landau frame (eqs. landau-lifshitz-*): eps U^a = T^{ab} U_b with
// U = gamma (1, ux, uy), as the fixed point
//   eps = T^00 - T^0i u_i,   u_i = (T^0i - T^ij u_j) / eps,
// started from the given (ux, uy) and stopped when |d eps| <= tol eps and
// |d u| <= tol (eps alone is insensitive to u where the momentum density is
// small).  Returns the iteration count (maxit + 1 if the cap was hit).
__device__ __forceinline__ int landau_solve(double T00, double T0x, double T0y, double Txx, double Txy,
                                            double Tyy, double tol, int maxit, double& eps, double& ux,
                                            double& uy) {
  double e = T00 - T0x * ux - T0y * uy;
  int it = 1;
  for (; it <= maxit; ++it) {
    const double inv = 1.0 / e;
    const double nx = (T0x - Txx * ux - Txy * uy) * inv;
    const double ny = (T0y - Txy * ux - Tyy * uy) * inv;
    const double du = fmax(fabs(nx - ux), fabs(ny - uy));
    ux = nx;
    uy = ny;
    const double en = T00 - T0x * ux - T0y * uy;
    const double de = fabs(en - e);
    e = en;
    if (de <= tol * e && du <= tol) break;
  }
  eps = e;
  return it;
}

// Projection coefficients b_k(U, T) of the unit-density Maxwell-Juttner
// distribution on the 10 in-plane second-order polynomials (Appendix B; T_R = 1
// so a_k = b_k).  From the moments int f p = U, int f p p = q U U - T eta,
// q = mbar K_3(z)/K_2(z) = zeta R + 4T, int f = R/zeta.
__device__ __forceinline__ void projections(const RlbmConsts& c, double T, double R, double U0, double Ux,
                                            double Uy, double b[RLBM_NB]) {
  const double b0 = R / c.zeta;
  const double q = fma(c.zeta, R, 4.0 * T);
  b[0] = b0;
  b[1] = (U0 - c.a1 * b0) * c.invA;
  b[2] = Ux * c.invB;
  b[3] = Uy * c.invB;
  b[4] = (q * U0 * U0 - T + c.c1 * U0 + c.c0 * b0) * c.inv_s3C;
  const double s = (q * U0 - c.d0) * c.invD;
  b[5] = s * Ux;
  b[6] = s * Uy;
  b[7] = q * Uy * Uy * (0.5 * c.invE);
  b[8] = q * (Uy * Uy - 2.0 * Ux * Ux) * (0.28867513459481288225 * c.invE);  // 1/(2 sqrt 3)
  b[9] = q * Ux * Uy * c.invE;
}

// Relaxation time per site from eta/s (Sec. IV): tau = 1/2 + (3/2)(eta/s) s hbar_c v0/(P dx)
// with s/P = (4 - ln(n/n_eq))/T in physical units, folded into tk1, tk2.
__device__ __forceinline__ double tau_eta_over_s(double tk1, double tk2, double n, double T) {
  return 0.5 + tk1 * (4.0 - log(tk2 * n / (T * T * T))) / T;
}

// Hardware dispatches workgroup b to XCD b % 8.  Give each XCD a contiguous
// range of logical tiles so neighbouring rows share an L2 (bijective for any nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + min(xcd, r) + k;
}

__device__ __forceinline__ int wrap_or_clamp(int s, int n, int bc, int small) {
  if (bc == RLBM_BC_PERIODIC) {
    if (small) return ((s % n) + n) % n;
    s += (s < 0) ? n : 0;
    s -= (s >= n) ? n : 0;
    return s;
  }
  return min(max(s, 0), n - 1);
}

}  // namespace rlbm
