// Per-site device mathematics of the relativistic lattice Boltzmann step
// (arXiv:1703.04605): Bessel ratio, equation of state inversion, Landau frame,
// projection coefficients.  All in float64.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/rlbm.h"
#include "bessel_ratio_coeffs.h"
#include "rlbm_tables.h"

namespace rlbm {

// The stencil table is read-only for the whole lifetime of every kernel;
// reading it through the constant address space lets uniform accesses become
// scalar loads through the scalar cache.
typedef const __attribute__((address_space(4))) RlbmTable* TabPtr;
__device__ __forceinline__ TabPtr as_tab(const RlbmTable* p) { return (TabPtr)p; }

// Quotients of the per-site chain: the hardware reciprocal (and reciprocal
// square root) refined by two Newton steps, each of which squares the relative
// error, then one residual correction of the product (a few ulp at most; the
// operands here are far from the overflow and underflow ranges that the
// library division guards against).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ double div_nr(double a, double d) {
  const double r = rcp_nr(d);
  const double q = a * r;
  return fma(fma(-d, q, a), r, q);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y * fma(-0.5 * x * y, y, 1.5);
}

// R(z) = K_1(z)/K_2(z), the Bessel ratio of the equation of state
// (eq. relativistic-eos).  For z < 1.5: the ascending series of K_0 and K_1
// (integer-order expansions with the logarithmic term, e.g. Abramowitz &
// Stegun 9.6.11/9.6.13) and K_2 = K_0 + 2 K_1/z; otherwise a Chebyshev
// expansion in t = 3/z - 1 (coefficients generated from mpmath).
__device__ __forceinline__ double k1k2_ratio(double z) {
  if (z < RLBM_BESSEL_Z_SPLIT) {
    // term ratios 1/k^2, 1/(k(k+1)) and the digamma sums 2 H_k + 1/(k+1) - 2 gamma
    constexpr double inv_k2[13] = {0, 1.0, 1.0 / 4, 1.0 / 9, 1.0 / 16, 1.0 / 25, 1.0 / 36, 1.0 / 49,
                                   1.0 / 64, 1.0 / 81, 1.0 / 100, 1.0 / 121, 1.0 / 144};
    constexpr double inv_kk1[13] = {0, 1.0 / 2, 1.0 / 6, 1.0 / 12, 1.0 / 20, 1.0 / 30, 1.0 / 42, 1.0 / 56,
                                    1.0 / 72, 1.0 / 90, 1.0 / 110, 1.0 / 132, 1.0 / 156};
    constexpr double euler_gamma = 0.57721566490153286061;
    double Hk[13], D1[13];
    Hk[0] = 0.0;
#pragma unroll
    for (int k = 1; k < 13; ++k) Hk[k] = Hk[k - 1] + 1.0 / (double)k;   // folded at compile time
#pragma unroll
    for (int k = 0; k < 13; ++k) D1[k] = 2.0 * Hk[k] + 1.0 / (double)(k + 1) - 2.0 * euler_gamma;
    const double y = 0.25 * z * z;
    double t0 = 1.0, t1 = 1.0;           // y^k/(k!)^2, y^k/(k!(k+1)!)
    double I0 = 1.0, I1s = 1.0;          // I0(z), 2 I1(z)/z
    double S0 = 0.0, S1 = D1[0];         // sum H_k t0_k, sum D1_k t1_k
#pragma unroll
    for (int k = 1; k < 13; ++k) {
      t0 *= y * inv_k2[k];
      t1 *= y * inv_kk1[k];
      I0 += t0;
      I1s += t1;
      S0 = fma(Hk[k], t0, S0);
      S1 = fma(D1[k], t1, S1);
    }
    const double L = log(0.5 * z);
    const double iz = 1.0 / z;
    const double K0 = S0 - (L + euler_gamma) * I0;
    const double K1 = iz + 0.5 * z * (L * I1s - 0.5 * S1);
    return K1 / fma(2.0 * iz, K1, K0);
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

// Inverse EOS from the per-stencil table: T = u g(u), u = e - zeta, with g a
// Chebyshev series on the quarter-octave of u (built on the host in long
// double from the same equation).  The table spans u in [2^-24, 2^24), i.e.
// T from about 4e-8 to 6e6 (in units of T_R); beyond it the site is flagged
// RLBM_H_EOS and T takes the limit of the equation of state (u = 3T/2 for
// T << mbar, u = 3T for T >> mbar).  The lanes of a wave are served one
// distinct piece at a time (the piece index is made uniform, so its
// coefficients come through scalar loads): smooth fields put a wave's sites in
// one or two pieces, and no vector memory access is needed.
__device__ __forceinline__ double eos_temperature_tab(TabPtr tb, double e, double zeta,
                                                     unsigned& flags) {
  const double u = e - zeta;
  int ex;
  const double m = frexp(u, &ex);          // u = m 2^ex, m in [1/2, 1)
  const int o = ex - 1 - RLBM_EOS_KMIN;
  const bool intab = u > 0.0 && o >= 0 && o < RLBM_EOS_NOCT;
  const double m2 = 2.0 * m;                // [1, 2)
  const int piece = min((int)((m2 - 1.0) * 4.0), 3);
  const double t = (m2 - 1.0 - 0.25 * piece) * 8.0 - 1.0;
  const int idx = intab ? o * 4 + piece : -1;
  const double t2 = 2.0 * t;
  double g = 0.0;
  bool todo = intab;
  for (unsigned long long pend = __builtin_amdgcn_ballot_w64(todo); pend != 0ull;
       pend = __builtin_amdgcn_ballot_w64(todo)) {
    const int iu = __builtin_amdgcn_readlane(idx, (int)__builtin_ctzll(pend));
    const __attribute__((address_space(4))) double* c = tb->eos[iu];
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = RLBM_EOS_DEG - 1; j >= 1; --j) {
      const double b0 = fma(t2, b1, c[j] - b2);
      b2 = b1;
      b1 = b0;
    }
    if (todo && idx == iu) {
      g = fma(t, b1, c[0] - b2);
      todo = false;
    }
  }
  if (!intab) {
    if (!(u > 0.0)) {
      flags |= RLBM_H_RANGE;
      return u * (1.0 / 1.5);
    }
    flags |= RLBM_H_EOS;
    return o < 0 ? u * (1.0 / 1.5) : u * (1.0 / 3.0);
  }
  return u * g;
}

// Landau frame by Newton's method on the characteristic polynomial of the
// mixed tensor: eps is the largest root of p(l) = det(l I - T eta), with
//   p(l) = (l - T00)[(l + Txx)(l + Tyy) - Txy^2] + T0x^2 (l + Tyy)
//          - 2 T0x T0y Txy + T0y^2 (l + Txx).
// T^00 bounds eps from above and p is increasing and convex to the right of
// its largest root, so iterates started at T^00 decrease monotonically (a
// start l0 below the root but above the inflection point of p jumps to the
// right of the root first).  The velocity then
// solves (eps delta_ij + T^ij) u_j = T^0i, the spatial rows of the eigenproblem.
// Stops one iteration after the step falls below `thresh` (quadratic
// convergence).  Returns the iteration count (maxit + 1 if the cap was hit).
__device__ __forceinline__ int landau_newton(double T00, double T0x, double T0y, double Txx, double Txy,
                                             double Tyy, double thresh, int maxit, double& eps, double& ux,
                                             double& uy, double l0) {
  double l = l0;
  const double b2c2 = T0x * T0x + T0y * T0y;
  const double bce2 = 2.0 * T0x * T0y * Txy;
  const double e2 = Txy * Txy;
  if (l != T00) {  // a start below T^00 must lie where p is increasing
    const double pd = l + Txx, pf = l + Tyy;
    if (!(fma(l - T00, pd + pf, fma(pd, pf, -e2) + b2c2) > 0.0)) l = T00;
  }
  int it = 1;
  bool done = false;
  for (; it <= maxit; ++it) {
    const double pd = l + Txx, pf = l + Tyy;
    const double m = fma(pd, pf, -e2);
    const double la = l - T00;
    const double p = fma(la, m, fma(T0x * T0x, pf, fma(T0y * T0y, pd, -bce2)));
    const double dp = fma(la, pd + pf, m + b2c2);
    const double step = div_nr(p, dp);
    l -= step;
    if (done) break;
    if (fabs(step) <= thresh * l) done = true;
  }
  const double pd = l + Txx, pf = l + Tyy;
  const double inv = rcp_nr(fma(pd, pf, -e2));
  ux = (T0x * pf - T0y * Txy) * inv;
  uy = (T0y * pd - T0x * Txy) * inv;
  eps = l;
  return it;
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
// Appendix A constants at mbar (T_R = 1) used by the projections.
struct ProjConsts {
  double zeta, inv_zeta, a1, invA, invB, c1, c0, inv_s3C, d0, invD, invE;
};

__device__ __forceinline__ ProjConsts proj_consts(TabPtr tb) {
  const auto& c = tb->c;
  return ProjConsts{c.zeta, c.inv_zeta, c.a1, c.invA, c.invB, c.c1, c.c0, c.inv_s3C, c.d0, c.invD, c.invE};
}

__device__ __forceinline__ void projections(const ProjConsts& c, double T, double R, double U0, double Ux,
                                            double Uy, double b[RLBM_NB]) {
  const double b0 = R * c.inv_zeta;
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

__device__ __forceinline__ void projections(TabPtr tb, double T, double R, double U0, double Ux, double Uy,
                                            double b[RLBM_NB]) {
  projections(proj_consts(tb), T, R, U0, Ux, Uy, b);
}

// Landau frame in 3D, by Newton's method on the characteristic polynomial of
// the 4 x 4 mixed tensor.  With S(l) = l I + T_s (T_s the spatial block of
// T^ab) and t = (T^0x, T^0y, T^0z), the block determinant gives
//   p(l) = det(l I - T eta) = (l - T00) det S(l) + t . adj(S(l)) t,
// and for a 3 x 3 matrix det S(l) = l^3 + e2 l^2 + e1 l + e0 and
// adj S(l) = l^2 I + l (e2 I - T_s) + adj(T_s), with e2 = tr T_s, e1 the sum
// of its principal 2 x 2 minors and e0 = det T_s.  The roots of p are real,
// so to the right of the largest one p and all its derivatives are positive
// and Newton from above (T^00 >= eps) decreases monotonically onto eps.  The
// velocity then solves the spatial rows (eps I + T_s) u = t:
// u = adj(S(eps)) t / det S(eps).  Returns the iteration count (maxit + 1 if
// the cap was hit).
__device__ __forceinline__ int landau_newton3(const double m[14], double thresh, int maxit, double& eps,
                                              double u[3], double l0) {
  // m: N0, Nx, Ny, Nz, T00, T0x, T0y, T0z, Txx, Txy, Txz, Tyy, Tyz, Tzz
  const double T00 = m[4], tx = m[5], ty = m[6], tz = m[7];
  const double xx = m[8], xy = m[9], xz = m[10], yy = m[11], yz = m[12], zz = m[13];
  const double axx = yy * zz - yz * yz, ayy = xx * zz - xz * xz, azz = xx * yy - xy * xy;
  const double axy = xz * yz - xy * zz, axz = xy * yz - xz * yy, ayz = xy * xz - xx * yz;
  const double e2 = xx + yy + zz, e1 = axx + ayy + azz, e0 = xx * axx + xy * axy + xz * axz;
  const double t2 = tx * tx + ty * ty + tz * tz;
  const double Ttx = xx * tx + xy * ty + xz * tz, Tty = xy * tx + yy * ty + yz * tz, Ttz = xz * tx + yz * ty + zz * tz;
  const double tTt = tx * Ttx + ty * Tty + tz * Ttz;
  const double Atx = axx * tx + axy * ty + axz * tz, Aty = axy * tx + ayy * ty + ayz * tz,
               Atz = axz * tx + ayz * ty + azz * tz;
  const double tAt = tx * Atx + ty * Aty + tz * Atz;
  const double c1 = e2 * t2 - tTt;
  double l = l0;
  if (l != T00) {  // a start below T^00 must lie where p is increasing and convex
    const double D = fma(fma(l + e2, l, e1), l, e0), Dp = fma(fma(3.0, l, 2.0 * e2), l, e1);
    const double dp = fma(l - T00, Dp, D) + fma(2.0 * t2, l, c1);
    if (!(dp > 0.0)) l = T00;
  }
  int it = 1;
  bool done = false;
  for (; it <= maxit; ++it) {
    const double D = fma(fma(l + e2, l, e1), l, e0);
    const double Dp = fma(fma(3.0, l, 2.0 * e2), l, e1);
    const double p = fma(l - T00, D, fma(fma(t2, l, c1), l, tAt));
    const double dp = fma(l - T00, Dp, D) + fma(2.0 * t2, l, c1);
    const double step = div_nr(p, dp);
    l -= step;
    if (done) break;
    if (fabs(step) <= thresh * l) done = true;
  }
  const double D = fma(fma(l + e2, l, e1), l, e0);
  const double inv = rcp_nr(D);
  // adj(S(eps)) t = eps^2 t + eps (e2 t - T_s t) + adj(T_s) t
  u[0] = fma(l, fma(l, tx, e2 * tx - Ttx), Atx) * inv;
  u[1] = fma(l, fma(l, ty, e2 * ty - Tty), Aty) * inv;
  u[2] = fma(l, fma(l, tz, e2 * tz - Ttz), Atz) * inv;
  eps = l;
  return it;
}

// Projection coefficients of all 14 polynomials (3D lattices; order of
// Appendix A: 0, 1_0, 1_x, 1_y, 1_z, 2_00, 2_0x, 2_0y, 2_0z, 2_xx, 2_yy,
// 2_xz, 2_yz, 2_xy, where 2_xx is (p_y^2 - p_z^2)/(2E) and 2_yy is
// (-2 p_x^2 + p_y^2 + p_z^2)/(2 sqrt 3 E)); the 2D set is these with U_z = 0.
__device__ __forceinline__ void projections3(const ProjConsts& c, double T, double R, double U0, const double U[3],
                                             double b[14]) {
  const double b0 = R * c.inv_zeta;
  const double q = fma(c.zeta, R, 4.0 * T);
  b[0] = b0;
  b[1] = (U0 - c.a1 * b0) * c.invA;
  b[2] = U[0] * c.invB;
  b[3] = U[1] * c.invB;
  b[4] = U[2] * c.invB;
  b[5] = (q * U0 * U0 - T + c.c1 * U0 + c.c0 * b0) * c.inv_s3C;
  const double s = (q * U0 - c.d0) * c.invD;
  b[6] = s * U[0];
  b[7] = s * U[1];
  b[8] = s * U[2];
  b[9] = q * (U[1] * U[1] - U[2] * U[2]) * (0.5 * c.invE);
  b[10] = q * (U[1] * U[1] + U[2] * U[2] - 2.0 * U[0] * U[0]) * (0.28867513459481288225 * c.invE);
  b[11] = q * U[0] * U[2] * c.invE;
  b[12] = q * U[1] * U[2] * c.invE;
  b[13] = q * U[0] * U[1] * c.invE;
}

// Relaxation time per site from eta/s (Sec. IV): tau = 1/2 + (3/2)(eta/s) s hbar_c v0/(P dx)
// with s/P = (4 - ln(n/n_eq))/T in physical units, folded into tk1, tk2.
__device__ __forceinline__ double tau_eta_over_s(double tk1, double tk2, double n, double T) {
  return 0.5 + tk1 * (4.0 - log(tk2 * n / (T * T * T))) / T;
}

// Third order: the 30 components (kO3Idx order) of the Maxwell-Juttner
// moment tensors int f^eq p^a .. p^c d^3p/p^0 of rank 0..3, density n
// included, U contravariant with U^0 = gamma.  With h = eps + P:
//   rank 0: (eps - 3P)/m^2          (n K_1/(m K_2), by the EOS)
//   rank 1: n U^a
//   rank 2: h U^a U^b - P eta^ab
//   rank 3: (n m^2 + 6 T h) U^a U^b U^c - T h (eta^ab U^c + eta^ac U^b + eta^bc U^a)
// The rank-3 scalars follow from the mass shell (the trace over one index
// pair is m^2 n U^c) and from the rest-frame <p0^2> of the distribution.
__device__ __forceinline__ constexpr double eta_ab(int a, int b) { return a != b ? 0.0 : (a == 0 ? 1.0 : -1.0); }

__device__ __forceinline__ void mj_moments_o3(double n, double eps, double P, double T, double inv_zeta,
                                              double zeta, const double U[4], double M[RLBM_NO3]) {
  const double h = eps + P;
  const double a3 = fma(6.0 * T, h, n * zeta * zeta), b3 = -T * h;
#pragma unroll
  for (int i = 0; i < RLBM_NO3; ++i) {
    const int a = kO3Idx[i][0], b = kO3Idx[i][1], c = kO3Idx[i][2];
    double v;
    if (a < 0)
      v = (eps - 3.0 * P) * inv_zeta * inv_zeta;
    else if (b < 0)
      v = n * U[a];
    else if (c < 0)
      v = h * U[a] * U[b] - P * eta_ab(a, b);
    else
      v = a3 * U[a] * U[b] * U[c] + b3 * (eta_ab(a, b) * U[c] + eta_ab(a, c) * U[b] + eta_ab(b, c) * U[a]);
    M[i] = v;
  }
}

// a_m = int f^eq q_m d^3p/p^0 for the centred, scaled monomials
// q_m = ((p0 - c)/s0)^k0 (p/sp)^(spatial part of m): the binomial expansion
// of (p0 - c)^k0 over the raw moments M (exponents and indices resolve at
// compile time).
__device__ __forceinline__ void centred_o3(const double M[RLBM_NO3], double c, double is0, double isp,
                                           double aq[RLBM_NO3]) {
#pragma unroll
  for (int m = 0; m < RLBM_NO3; ++m) {
    const int k0 = o3_exp(m, 0), ks = o3_exp(m, 1) + o3_exp(m, 2) + o3_exp(m, 3);
    const double m0 = M[kO3Raw.r[m][0]];
    double v;
    if (k0 == 0) {
      v = m0;
    } else if (k0 == 1) {
      v = fma(-c, m0, M[kO3Raw.r[m][1]]);
    } else if (k0 == 2) {
      v = fma(c * c, m0, fma(-2.0 * c, M[kO3Raw.r[m][1]], M[kO3Raw.r[m][2]]));
    } else {
      v = fma(-c * c * c, m0, fma(3.0 * c * c, M[kO3Raw.r[m][1]], fma(-3.0 * c, M[kO3Raw.r[m][2]], M[kO3Raw.r[m][3]])));
    }
    double sc = 1.0;
#pragma unroll
    for (int e = 0; e < k0; ++e) sc *= is0;
#pragma unroll
    for (int e = 0; e < ks; ++e) sc *= isp;
    aq[m] = v * sc;
  }
}

// Hardware dispatches workgroup b to XCD b % 8.  Give each XCD a contiguous
// range of logical tiles so neighbouring rows share an L2 (bijective for any nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + min(xcd, r) + k;
}

}  // namespace rlbm
