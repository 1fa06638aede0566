// Host-side construction of the quadrature stencil and of the population-class
// table (Sec. III.A-D of arXiv:1703.04605), in long double.  No HIP calls.
//
//  * Bessel functions K_nu(x) from the integral representation
//    K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (trapezoid rule, which is
//    spectrally accurate for this even, entire integrand).
//  * Energy moments of the weight function omega(p0) = exp(-p0)/N_R
//    (eq. mj-poly-weighting-factor, T_R = 1) in the variable p0 = m cosh t,
//    where d^3p/p^0 = 4 pi m^2 sinh^2 t dt dOmega/(4 pi).
//  * Weights: for full-symmetric groups the second-order conditions of
//    eq. ortho1 reduce to six linear equations in the group weights: the
//    energy moments sum_k N_k w_k (p0_k)^a = mu_a, a = 0..4, and the quartic
//    isotropy sum_k w_k sum_{i in k} (p_x^4 - 3 p_x^2 p_y^2) = 0.
//    All 14 x 14 conditions are then verified explicitly.
//  * Classes: the 1-thick lattice (Sec. IV: 1 x N x M and 1 x 1 x N) lets
//    populations of one group with equal in-plane displacement be merged
//    exactly, because they share p^0, the in-plane momentum and (U_z = 0)
//    their relaxation frequency.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <memory>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "../../include/rlbm.h"
#include "rlbm_stencil.h"

typedef long double ld;

namespace {

// exp(x) K_nu(x) = int_0^inf exp(-x (cosh t - 1)) cosh(nu t) dt.  Only ratios
// of K's at one argument are ever used, so the scaled form avoids underflow.
ld besselk_scaled_ld(int nu, ld x) {
  // Trapezoid rule: for this entire integrand the error decays like
  // exp(-pi^2/h), and near t = 0 it is a Gaussian of width 1/sqrt(x), so h is
  // also kept below half that width.
  const ld h = std::min(1.0L / 8.0L, 0.5L / sqrtl(x));
  ld s = 0.5L;
  for (int k = 1; k < 100000; ++k) {
    ld t = k * h;
    ld ch = coshl(t);
    ld v = expl(-x * (ch - 1.0L)) * coshl(nu * t);
    s += v;
    if (x * (ch - 1.0L) > 60.0L + nu * t && v < 1e-22L * s) break;
  }
  return s * h;
}

// S_a = int_0^inf exp(-m (cosh t - 1)) cosh^a t sinh^2 t dt, a = 0..4
void energy_integrals(ld m, ld S[5]) {
  const ld h = std::min(1.0L / 8.0L, 0.5L / sqrtl(m));
  for (int a = 0; a < 5; ++a) S[a] = 0.0L;
  for (int k = 1; k < 200000; ++k) {
    ld t = k * h;
    ld c = coshl(t), sh = sinhl(t);
    ld e = expl(-m * (c - 1.0L)) * sh * sh;
    ld p = 1.0L;
    for (int a = 0; a < 5; ++a) {
      S[a] += e * p;
      p *= c;
    }
    if (m * (c - 1.0L) > 60.0L) break;
  }
}

struct Pop {
  int g;
  int n[3];
};

std::vector<std::array<int, 3>> fs_orbit(const int b[3]) {
  int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::set<std::array<int, 3>> s;
  for (auto& p : perm)
    for (int sg = 0; sg < 8; ++sg) {
      std::array<int, 3> v;
      for (int a = 0; a < 3; ++a) v[a] = ((sg >> a) & 1 ? -1 : 1) * b[p[a]];
      s.insert(v);
    }
  return std::vector<std::array<int, 3>>(s.begin(), s.end());
}

struct Basis {
  ld m, k1, k2, k3;
  ld A, B, C, D, E, a1, c1, c0, d0;
  explicit Basis(ld mbar) : m(mbar) {
    k1 = besselk_scaled_ld(1, m);   // common factor exp(-m) cancels in every ratio below
    k2 = besselk_scaled_ld(2, m);
    k3 = besselk_scaled_ld(3, m);
    ld den = m * k1 * k1 + 3 * k2 * k1 - m * k2 * k2;
    A = sqrtl(m * (m + k2 * (3 * k1 - m * k2) / (k1 * k1)));
    B = sqrtl(m * k2 / k1);
    C = sqrtl(2 * m * m + 5 * m * k2 / k1 - 3 * k1 * (m * k1 + 3 * k2) / den + 3);
    D = sqrtl(m * m * (m * k2 * k2 + 5 * k3 * k2 - m * k3 * k3) / (k1 * k2));
    E = sqrtl(m * m * k3 / k1);
    a1 = m * k2 / k1;
    c1 = 3 / (-m * k1 / k2 + m * k2 / k1 - 3) - 3;
    c0 = 3 * k1 * (m * k1 + 3 * k2) / den - m * m - 3;
    d0 = m * k3 / k2;
  }
  // all 14 second-order polynomials of Appendix A at p = (p0, px, py, pz)
  void eval14(const ld p[4], ld J[14]) const {
    const ld s3 = sqrtl(3.0L);
    ld p0 = p[0], x = p[1], y = p[2], z = p[3];
    J[0] = 1;
    J[1] = (p0 - a1) / A;
    J[2] = x / B;
    J[3] = y / B;
    J[4] = z / B;
    J[5] = (p0 * p0 + c1 * p0 + c0) / (s3 * C);
    J[6] = x * (p0 - d0) / D;
    J[7] = y * (p0 - d0) / D;
    J[8] = z * (p0 - d0) / D;
    J[9] = (y * y - z * z) / (2 * E);
    J[10] = (-2 * x * x + y * y + z * z) / (2 * s3 * E);
    J[11] = x * z / E;
    J[12] = y * z / E;
    J[13] = x * y / E;
  }
};

// index of the 10 in-plane polynomials among the 14
const int kInPlane[RLBM_NB] = {0, 1, 2, 3, 5, 6, 7, 9, 10, 13};

bool solve_dense(int n, std::vector<ld> a, std::vector<ld> b, std::vector<ld>& x) {
  // Gaussian elimination with partial pivoting, a row-major n x n
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(a[r * n + c]) > fabsl(a[piv * n + c])) piv = r;
    if (a[piv * n + c] == 0.0L) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(a[c * n + k], a[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      ld f = a[r * n + c] / a[c * n + c];
      for (int k = c; k < n; ++k) a[r * n + k] -= f * a[c * n + k];
      b[r] -= f * b[c];
    }
  }
  x.assign(n, 0.0L);
  for (int r = n - 1; r >= 0; --r) {
    ld s = b[r];
    for (int k = r + 1; k < n; ++k) s -= a[r * n + k] * x[k];
    x[r] = s / a[r * n + r];
  }
  return true;
}

struct Stencil {
  ld m;
  int ng;
  std::vector<std::array<int, 3>> base;
  std::vector<std::vector<std::array<int, 3>>> orbit;
  std::vector<int> n2;
  ld mu[5];
  ld vmax;

  Stencil(ld mbar, int n_groups, const int* gb) : m(mbar), ng(n_groups) {
    int maxn2 = 0;
    for (int g = 0; g < ng; ++g) {
      std::array<int, 3> b = {gb[3 * g], gb[3 * g + 1], gb[3 * g + 2]};
      base.push_back(b);
      orbit.push_back(fs_orbit(b.data()));
      n2.push_back(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      maxn2 = std::max(maxn2, n2.back());
    }
    vmax = maxn2 > 0 ? 1.0L / sqrtl((ld)maxn2) : 1.0L;
    ld S[5];
    energy_integrals(m, S);
    ld p = 1.0L;
    for (int a = 0; a < 5; ++a) {
      mu[a] = p * S[a] / S[0];
      p *= m;
    }
  }

  // the six reduced conditions as a 6 x 6 system a w = b (row-major a)
  void system(ld v0, std::vector<ld>& a, std::vector<ld>& b) const {
    a.assign(36, 0.0L);
    b.assign(6, 0.0L);
    for (int g = 0; g < 6; ++g) {
      ld gam = 1.0L / sqrtl(1.0L - v0 * v0 * n2[g]);
      ld p0 = m * gam;
      ld N = (ld)orbit[g].size();
      ld pw = 1.0L;
      for (int r = 0; r < 5; ++r) {
        a[r * 6 + g] = N * pw;
        pw *= p0;
      }
      ld iso = 0.0L;
      for (auto& v : orbit[g]) iso += (ld)v[0] * v[0] * v[0] * v[0] - 3.0L * v[0] * v[0] * v[1] * v[1];
      ld pm = m * gam * v0;
      a[5 * 6 + g] = iso * pm * pm * pm * pm;
    }
    for (int r = 0; r < 5; ++r) b[r] = mu[r];
    b[5] = 0.0L;
  }

  // the six reduced conditions; returns false if singular
  bool weights(ld v0, std::vector<ld>& w) const {
    if (ng != 6) return false;
    std::vector<ld> a, b;
    system(v0, a, b);
    return solve_dense(6, a, b, w);
  }


  ld min_weight(ld v0) const {
    std::vector<ld> w;
    if (!weights(v0, w)) return -1e300L;
    ld mn = w[0];
    for (ld x : w) mn = std::min(mn, x);
    return mn;
  }

  void populations(ld v0, std::vector<Pop>& pops, std::vector<std::array<ld, 4>>& mom) const {
    pops.clear();
    mom.clear();
    for (int g = 0; g < ng; ++g) {
      ld gam = 1.0L / sqrtl(1.0L - v0 * v0 * n2[g]);
      for (auto& v : orbit[g]) {
        pops.push_back({g, {v[0], v[1], v[2]}});
        mom.push_back({m * gam, m * gam * v0 * v[0], m * gam * v0 * v[1], m * gam * v0 * v[2]});
      }
    }
  }
};

// Eigenvalues of a symmetric n x n matrix (cyclic Jacobi rotations).
void jacobi_eigenvalues(int n, std::vector<ld> a, std::vector<ld>& ev) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    ld off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-60L) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const ld apq = a[p * n + q];
        if (apq == 0) continue;
        const ld theta = (a[q * n + q] - a[p * n + p]) / (2 * apq);
        const ld t = (theta >= 0 ? 1 : -1) / (fabsl(theta) + sqrtl(theta * theta + 1));
        const ld c = 1 / sqrtl(t * t + 1), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const ld akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - sn * akq;
          a[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const ld apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - sn * aqk;
          a[q * n + k] = sn * apk + c * aqk;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = a[i * n + i];
}

void set_err(char* err, size_t len, const char* msg) {
  if (err && len) snprintf(err, len, "%s", msg);
}

// ---- third order (Sec. III.A, III.D) ----

// R[j][s] = <p0^j |p|^s> under omega (s even, angular part excluded), j, s <= 6:
// m^(j+s) S(j, s) / S(0, 0) with S(j, s) = int exp(-m (cosh t - 1))
// cosh^j t sinh^(2+s) t dt (trapezoid rule; the integrand is even in t).
void omega_radial_moments(ld m, ld R[7][7]) {
  const ld h = std::min(1.0L / 8.0L, 0.5L / sqrtl(m));
  ld S[7][7] = {};
  for (int k = 0; k < 400000; ++k) {
    const ld t = k * h, c = coshl(t), sh = sinhl(t);
    const ld e = expl(-m * (c - 1.0L)) * sh * sh * (k == 0 ? 0.5L : 1.0L);
    ld cj = 1.0L;
    for (int j = 0; j < 7; ++j) {
      ld ss = 1.0L;
      for (int q = 0; q < 7; ++q) {
        S[j][q] += e * cj * ss;
        ss *= sh;
      }
      cj *= c;
    }
    if (m * (c - 1.0L) > 90.0L + 13.0L * t) break;
  }
  for (int j = 0; j < 7; ++j)
    for (int q = 0; q < 7; ++q) R[j][q] = powl(m, (ld)(j + q)) * S[j][q] / S[0][0];
}

// <n_x^a n_y^b n_z^c> over the unit sphere: (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!!
// for even exponents, 0 otherwise
ld sphere_avg(int a, int b, int c) {
  if ((a | b | c) & 1) return 0.0L;
  auto dfact = [](int n) {
    ld r = 1.0L;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
  };
  return dfact(a - 1) * dfact(b - 1) * dfact(c - 1) / dfact(a + b + c + 1);
}

// exponents (k0, kx, ky, kz) of monomial m of the third-order list
void o3_exponents(int mono, int e[4]) {
  e[0] = e[1] = e[2] = e[3] = 0;
  for (int r = 0; r < 3; ++r)
    if (kO3Idx[mono][r] >= 0) ++e[kO3Idx[mono][r]];
}

struct Stencil3 {
  ld m;
  int ng;
  std::vector<std::vector<std::array<int, 3>>> orbit;
  std::vector<int> n2;
  ld R[7][7];
  ld vmax;
  ld rhs[11];
  ld c = 0, s = 1, sp = 1;  // centre and spread of p0, rms of p_x

  Stencil3(ld mbar, int n_groups, const int* gb) : m(mbar), ng(n_groups) {
    int maxn2 = 0;
    for (int g = 0; g < ng; ++g) {
      const int b[3] = {gb[3 * g], gb[3 * g + 1], gb[3 * g + 2]};
      orbit.push_back(fs_orbit(b));
      n2.push_back(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
      maxn2 = std::max(maxn2, n2.back());
    }
    vmax = maxn2 > 0 ? 1.0L / sqrtl((ld)maxn2) : 1.0L;
    omega_radial_moments(m, R);
    // The conditions are written in the centred, scaled energy
    // t = (p0 - c)/s and momentum p/sp (c = <p0>, s its spread, sp^2 = <p_x^2>):
    // exact integrals of t^j (j <= 6), t^j (p_x/sp)^4 (j <= 2) and
    // (p_x p_y p_z / sp^3)^2.  They are combinations of the conditions on
    // p0^j, p0^j p_x^4 and p_x^2 p_y^2 p_z^2 (same solution), far better
    // conditioned than raw powers of p0 at large mbar.
    c = R[1][0];
    s = sqrtl(R[2][0] - c * c);
    sp = sqrtl(R[0][2] / 3.0L);
    auto tmom = [this](int j, int k) {  // <t^j |p|^k>
      ld sum = 0, bin = 1;
      for (int i = 0; i <= j; ++i) {
        sum += bin * powl(-c, (ld)(j - i)) * R[i][k];
        bin = bin * (j - i) / (i + 1);
      }
      return sum / powl(s, (ld)j);
    };
    for (int j = 0; j < 7; ++j) rhs[j] = tmom(j, 0);
    for (int j = 0; j < 3; ++j) rhs[7 + j] = tmom(j, 4) * sphere_avg(4, 0, 0) / powl(sp, 4.0L);
    rhs[10] = R[0][6] * sphere_avg(2, 2, 2) / powl(sp, 6.0L);
  }

  // the eleven conditions as a square system in the per-population weights
  bool weights(ld v0, std::vector<ld>& w) const {
    if (ng != 11) return false;
    std::vector<ld> a(121, 0.0L), b(rhs, rhs + 11);
    for (int g = 0; g < 11; ++g) {
      const ld gam = 1.0L / sqrtl(1.0L - v0 * v0 * n2[g]);
      const ld t = (m * gam - c) / s, pm = m * gam * v0 / sp;
      ld pw = 1.0L;
      for (int j = 0; j < 7; ++j) {
        a[j * 11 + g] = (ld)orbit[g].size() * pw;
        pw *= t;
      }
      ld x4 = 0, x2y2z2 = 0;
      for (auto& v : orbit[g]) {
        x4 += (ld)v[0] * v[0] * v[0] * v[0];
        x2y2z2 += (ld)v[0] * v[0] * v[1] * v[1] * v[2] * v[2];
      }
      const ld pm4 = pm * pm * pm * pm;
      for (int j = 0; j < 3; ++j) a[(7 + j) * 11 + g] = x4 * pm4 * powl(t, (ld)j);
      a[10 * 11 + g] = x2y2z2 * pm4 * pm * pm;
    }
    return solve_dense(11, a, b, w);
  }

  ld min_weight(ld v0) const {
    std::vector<ld> w;
    if (!weights(v0, w)) return -1e300L;
    return *std::min_element(w.begin(), w.end());
  }
};

// Cholesky factor (lower) of a symmetric positive definite n x n matrix
bool cholesky(int n, const std::vector<ld>& a, std::vector<ld>& L) {
  L.assign(n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      ld s = a[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      if (i == j) {
        if (!(s > 0)) return false;
        L[i * n + i] = sqrtl(s);
      } else {
        L[i * n + j] = s / L[j * n + j];
      }
    }
  return true;
}

}  // namespace

// The interval of v0 in the description's search range on which every
// weight is positive: grid search for the v0 that maximises the smallest
// weight (zooming in until it is positive), edges bracketed by doubling steps
// and bisected, then a check that the interval is one connected run.
template <class MinW>
int positive_window(const MinW& minw, ld vmax, const rlbm_stencil_desc* d, ld& wlo, ld& whi, char* err,
                    size_t errlen) {
  // search the interval of all-positive weights: grid, zoom on max min_k w_k, bisect edges
  ld lo = d->v0_lo > 0 ? (ld)d->v0_lo : 1e-6L;
  ld hi = d->v0_hi > 0 ? std::min((ld)d->v0_hi, vmax * (1 - 1e-12L)) : vmax * (1 - 1e-12L);
  if (!(hi > lo)) {
    set_err(err, errlen, "empty v0 search interval");
    return RLBM_EINVAL;
  }
  const int G = 400;
  ld a = lo, b = hi, best = lo, bestv = -1e300L;
  for (int zoom = 0; zoom < 14 && bestv <= 0; ++zoom) {
    ld step = (b - a) / G;
    for (int i = 0; i <= G; ++i) {
      ld v = a + step * i;
      ld mw = minw(v);
      if (mw > bestv) {
        bestv = mw;
        best = v;
      }
    }
    a = std::max(best - 2 * step, lo);
    b = std::min(best + 2 * step, hi);
  }
  if (!(bestv > 0)) {
    set_err(err, errlen, "no v0 with all weights positive in the search interval");
    return RLBM_ENOSTENCIL;
  }
  // bracket each edge by steps that double from the last grid spacing (after
  // deep zooming that spacing can be far below the window's width), then bisect
  const ld step0 = std::max((b - a) / G, (hi - lo) * 1e-15L);
  ld l_in = best, l_out = lo, r_in = best, r_out = hi;
  for (ld s = step0; best - s > lo; s *= 2) {
    if (minw(best - s) > 0) {
      l_in = best - s;
    } else {
      l_out = best - s;
      break;
    }
  }
  for (ld s = step0; best + s < hi; s *= 2) {
    if (minw(best + s) > 0) {
      r_in = best + s;
    } else {
      r_out = best + s;
      break;
    }
  }
  auto bisect = [&minw](ld& in, ld& out) {
    for (int it = 0; it < 100; ++it) {
      const ld mid = 0.5L * (in + out);
      if (minw(mid) > 0) in = mid; else out = mid;
    }
  };
  bisect(l_in, l_out);
  bisect(r_in, r_out);
  // A doubled step can jump over a run of negative weights into another
  // positive run; the window must be the run that holds `best`.  Sample it:
  // if any interior point is not positive, walk out from `best` at the
  // finest spacing instead (bounded), and bisect from there.
  auto connected = [&minw](ld x0, ld x1) {
    for (int i = 1; i < 64; ++i)
      if (!(minw(x0 + (x1 - x0) * i / 64) > 0)) return false;
    return true;
  };
  if (!connected(l_in, best) || !connected(best, r_in)) {
    // (a walk that ends without leaving the run keeps its last point as the
    // edge: out == in leaves nothing to bisect)
    l_in = best, r_in = best;
    l_out = lo, r_out = hi;
    bool l_found = false, r_found = false;
    for (int i = 1; i <= 100000 && best - i * step0 > lo; ++i) {
      if (minw(best - i * step0) > 0) {
        l_in = best - i * step0;
      } else {
        l_out = best - i * step0;
        l_found = true;
        break;
      }
    }
    for (int i = 1; i <= 100000 && best + i * step0 < hi; ++i) {
      if (minw(best + i * step0) > 0) {
        r_in = best + i * step0;
      } else {
        r_out = best + i * step0;
        r_found = true;
        break;
      }
    }
    if (l_found) bisect(l_in, l_out);
    if (r_found) bisect(r_in, r_out);
  }
  wlo = l_in;
  whi = r_in;
  return RLBM_OK;
}

// Bessel ratio K1/K2 in long double (host reference state only)
static ld k1k2_ld(ld z) { return besselk_scaled_ld(1, z) / besselk_scaled_ld(2, z); }

// Third-order quadrature and tables (float64 storage only).  The continuous
// Gram matrix is taken over a centred, scaled copy q of the 30 monomials,
// q_m = ((p0 - c)/s0)^k0 (p_x/sp)^kx (p_y/sp)^ky (p_z/sp)^kz with c = <p0>,
// s0 its spread and sp^2 = <p_x^2> (well conditioned at every mbar);
// orthonormal polynomials are J = L^-1 q with G_q = L L^T.  The equilibrium
// f_i = n w_i sum_k a_k J_k(p_i) with a = L^-1 int f^eq q becomes
// f_i = R_i . a, with a = int f^eq q d^3p/p^0 (formed on the device from
// the raw moment tensors) and R_i = w_i L^-T J(p_i).
static int build_table_o3(const rlbm_stencil_desc* d, rlbm_stencil_info* info, RlbmTable* tab, char* err,
                          size_t errlen) {
  if (d->n_groups != 11 || (d->precision != RLBM_FP64 && d->precision != RLBM_FP32_DEV)) {
    set_err(err, errlen, "third order needs 11 groups and float64 or float32-deviation storage");
    return RLBM_EINVAL;
  }
  Stencil3 st((ld)d->zeta, d->n_groups, d->group_base);
  for (int g = 0; g < 11; ++g)
    for (int h = g + 1; h < 11; ++h)
      if (st.orbit[g] == st.orbit[h]) {
        set_err(err, errlen, "repeated velocity group");
        return RLBM_EINVAL;
      }
  ld v0 = d->v0;
  ld wlo = 0, whi = 0;
  if (d->weights && !(v0 > 0)) {
    set_err(err, errlen, "given weights need a given v0");
    return RLBM_EINVAL;
  }
  if (!(v0 > 0)) {
    const int rc = positive_window([&st](ld v) { return st.min_weight(v); }, st.vmax, d, wlo, whi, err, errlen);
    if (rc) return rc;
    v0 = 0.5L * (wlo + whi);
  }
  if (!(v0 < st.vmax)) {
    set_err(err, errlen, "v0 too large: a group would move faster than light");
    return RLBM_EINVAL;
  }
  std::vector<ld> w(11);
  if (d->weights) {
    for (int g = 0; g < 11; ++g) w[g] = (ld)d->weights[g];
  } else if (!st.weights(v0, w)) {
    set_err(err, errlen, "singular quadrature system for this group set");
    return RLBM_ENOSTENCIL;
  }
  for (ld x : w)
    if (!(x > 0)) {
      set_err(err, errlen, "quadrature weights not all positive at this v0");
      return RLBM_ENOSTENCIL;
    }

  // centred, scaled basis and its continuous Gram matrix
  const ld m = (ld)d->zeta;
  const ld c0 = st.R[1][0], s0 = sqrtl(st.R[2][0] - c0 * c0), sp = sqrtl(st.R[0][2] / 3.0L);
  int ex[RLBM_NO3][4];
  for (int a = 0; a < RLBM_NO3; ++a) o3_exponents(a, ex[a]);
  auto binom = [](int n, int k) {
    ld r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  // B[a][r]: coefficient of raw monomial r in q_a
  std::vector<ld> B(RLBM_NO3 * RLBM_NO3, 0.0L);
  for (int a = 0; a < RLBM_NO3; ++a)
    for (int r = 0; r < RLBM_NO3; ++r) {
      if (ex[r][1] != ex[a][1] || ex[r][2] != ex[a][2] || ex[r][3] != ex[a][3] || ex[r][0] > ex[a][0]) continue;
      const int K = ex[a][0], k = ex[r][0];
      B[a * RLBM_NO3 + r] = binom(K, k) * powl(-c0, (ld)(K - k)) /
                            (powl(s0, (ld)K) * powl(sp, (ld)(ex[a][1] + ex[a][2] + ex[a][3])));
    }
  std::vector<ld> G(RLBM_NO3 * RLBM_NO3, 0.0L);
  for (int a = 0; a < RLBM_NO3; ++a)
    for (int b = 0; b < RLBM_NO3; ++b) {
      ld sum = 0;
      for (int r = 0; r < RLBM_NO3; ++r) {
        const ld br = B[a * RLBM_NO3 + r];
        if (br == 0) continue;
        for (int t = 0; t < RLBM_NO3; ++t) {
          const ld bt = B[b * RLBM_NO3 + t];
          if (bt == 0) continue;
          const int e0 = ex[r][0] + ex[t][0], ex_ = ex[r][1] + ex[t][1], ey = ex[r][2] + ex[t][2],
                    ez = ex[r][3] + ex[t][3];
          sum += br * bt * st.R[e0][ex_ + ey + ez] * sphere_avg(ex_, ey, ez);
        }
      }
      G[a * RLBM_NO3 + b] = sum;
    }
  std::vector<ld> L;
  if (!cholesky(RLBM_NO3, G, L)) {
    set_err(err, errlen, "third-order Gram matrix not positive definite");
    return RLBM_EINVAL;
  }
  auto lower_solve = [&L](const ld* y, ld* x) {  // x = L^-1 y
    for (int i = 0; i < RLBM_NO3; ++i) {
      ld s = y[i];
      for (int k = 0; k < i; ++k) s -= L[i * RLBM_NO3 + k] * x[k];
      x[i] = s / L[i * RLBM_NO3 + i];
    }
  };
  auto upper_solve = [&L](const ld* y, ld* x) {  // x = L^-T y
    for (int i = RLBM_NO3 - 1; i >= 0; --i) {
      ld s = y[i];
      for (int k = i + 1; k < RLBM_NO3; ++k) s -= L[k * RLBM_NO3 + i] * x[k];
      x[i] = s / L[i * RLBM_NO3 + i];
    }
  };

  // populations and their orthonormal polynomial values
  struct P3 { int g; int n[3]; ld p[4]; };
  std::vector<P3> pops;
  for (int g = 0; g < 11; ++g) {
    const ld gam = 1.0L / sqrtl(1.0L - v0 * v0 * st.n2[g]);
    for (auto& v : st.orbit[g])
      pops.push_back({g, {v[0], v[1], v[2]}, {m * gam, m * gam * v0 * v[0], m * gam * v0 * v[1], m * gam * v0 * v[2]}});
  }
  const int np = (int)pops.size();
  std::vector<std::array<ld, RLBM_NO3>> J(np);
  for (int i = 0; i < np; ++i) {
    ld raw[RLBM_NO3], q[RLBM_NO3];
    for (int r = 0; r < RLBM_NO3; ++r) {
      ld v = 1;
      for (int k = 0; k < 3; ++k)
        if (kO3Idx[r][k] >= 0) v *= pops[i].p[kO3Idx[r][k]];
      raw[r] = v;
    }
    for (int a = 0; a < RLBM_NO3; ++a) {
      ld sum = 0;
      for (int r = 0; r < RLBM_NO3; ++r) sum += B[a * RLBM_NO3 + r] * raw[r];
      q[a] = sum;
    }
    lower_solve(q, J[i].data());
  }
  // orthonormality of the 30 polynomials under the quadrature (eq. ortho2)
  ld res = 0;
  for (int l = 0; l < RLBM_NO3; ++l)
    for (int k = l; k < RLBM_NO3; ++k) {
      ld sum = 0;
      for (int i = 0; i < np; ++i) sum += w[pops[i].g] * J[i][l] * J[i][k];
      res = std::max(res, fabsl(sum - (l == k ? 1.0L : 0.0L)));
    }
  // condition number of the quadrature problem's system matrix (465 x 11)
  ld cond = INFINITY;
  {
    std::vector<ld> AtA(121, 0.0L), row(11);
    for (int l = 0; l < RLBM_NO3; ++l)
      for (int k = l; k < RLBM_NO3; ++k) {
        std::fill(row.begin(), row.end(), 0.0L);
        for (int i = 0; i < np; ++i) row[pops[i].g] += J[i][l] * J[i][k];
        for (int g = 0; g < 11; ++g)
          for (int h = 0; h < 11; ++h) AtA[g * 11 + h] += row[g] * row[h];
      }
    std::vector<ld> ev;
    jacobi_eigenvalues(11, AtA, ev);
    const ld mx = *std::max_element(ev.begin(), ev.end()), mn = *std::min_element(ev.begin(), ev.end());
    if (mn > 0) cond = sqrtl(mx / mn);
  }
  if (!(res < 1e-10L)) {
    set_err(err, errlen, "third-order orthonormality conditions not satisfied by this group set");
    return RLBM_ENOSTENCIL;
  }

  // classes as at second order
  std::map<std::tuple<int, int, int, int>, int> key2class;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < np; ++i) {
    auto key = std::make_tuple(pops[i].g, pops[i].n[0], d->dim >= 2 ? pops[i].n[1] : 0,
                               d->dim == 3 ? pops[i].n[2] : 0);
    auto it = key2class.find(key);
    if (it == key2class.end()) {
      key2class[key] = (int)members.size();
      members.push_back({i});
    } else {
      members[it->second].push_back(i);
    }
  }
  const int Q = (int)members.size();
  if (Q > RLBM_QMAX) {
    set_err(err, errlen, "stencil has more population classes than the library supports");
    return RLBM_EINVAL;
  }
  int sx_max = 0, sy_max = 0, sz_max = 0;
  for (auto& p : pops) {
    sx_max = std::max(sx_max, abs(p.n[0]));
    if (d->dim >= 2) sy_max = std::max(sy_max, abs(p.n[1]));
    if (d->dim == 3) sz_max = std::max(sz_max, abs(p.n[2]));
  }
  const int max_shift = std::max(sx_max, std::max(sy_max, sz_max));
  if (max_shift > 16) {
    set_err(err, errlen, "displacements above 16 lattice sites are not supported");
    return RLBM_EINVAL;
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->q3 = np;
    info->q = Q;
    info->v0 = (double)v0;
    info->v0_lo = (double)wlo;
    info->v0_hi = (double)whi;
    for (int g = 0; g < 11; ++g) info->weights[g] = (double)w[g];
    info->ortho_residual = (double)res;
    info->max_shift = max_shift;
    info->cond = (double)cond;
  }
  if (!tab) return RLBM_OK;

  memset(tab, 0, sizeof(*tab));
  RlbmConsts& c = tab->c;
  c.Q = Q;
  c.order = 3;
  c.dim = d->dim;
  c.precision = d->precision;
  c.max_shift = max_shift;
  c.sx_max = sx_max;
  c.sy_max = sy_max;
  c.sz_max = sz_max;
  c.zeta = d->zeta;
  c.inv_zeta = (double)(1.0L / m);
  c.v0 = (double)v0;
  c.n_ref = 1.0;
  c.T_ref = 1.0;
  c.o3_c = (double)c0;
  c.o3_is0 = (double)(1.0L / s0);
  c.o3_isp = (double)(1.0L / sp);
  for (int j = 0; j < Q; ++j) {
    const P3& p0 = pops[members[j][0]];
    tab->nx[j] = p0.n[0];
    tab->ny[j] = d->dim >= 2 ? p0.n[1] : 0;
    tab->nz[j] = d->dim == 3 ? p0.n[2] : 0;
    tab->dnx[j] = tab->nx[j];
    tab->dny[j] = tab->ny[j];
    tab->p0[j] = (double)p0.p[0];
    tab->px[j] = (double)p0.p[1];
    tab->py[j] = d->dim >= 2 ? (double)p0.p[2] : 0.0;
    tab->pz[j] = d->dim == 3 ? (double)p0.p[3] : 0.0;
    // equilibrium row in the q basis: sum over the class of w_i L^-T J(p_i)
    ld row[RLBM_NO3] = {};
    for (int i : members[j]) {
      ld y[RLBM_NO3];
      upper_solve(J[i].data(), y);
      for (int r = 0; r < RLBM_NO3; ++r) row[r] += w[pops[i].g] * y[r];
    }
    const O3Act& act = kO3Act[d->dim];
    for (int r = 0; r < act.n; ++r) tab->rowo3[j][r] = (double)row[(int)act.m[r]];
    tab->rowo3[j][RLBM_RO3_NX] = tab->nx[j];
    tab->rowo3[j][RLBM_RO3_NY] = tab->ny[j];
    tab->rowo3[j][RLBM_RO3_NZ] = tab->nz[j];
    // moment rows of the 3D kernels.  The members of a merged class carry
    // equal populations (the flow has no velocity along the merged axes and
    // does not vary along them), so odd moments in the merged components
    // cancel over the class and its squared components enter as the members'
    // mean
    const ld px = p0.p[1], py = d->dim >= 2 ? p0.p[2] : 0.0L, pz = d->dim == 3 ? p0.p[3] : 0.0L;
    const ld e = p0.p[0];
    ld pyy = 0, pzz = 0;
    for (int i : members[j]) {
      pyy += pops[i].p[2] * pops[i].p[2];
      pzz += pops[i].p[3] * pops[i].p[3];
    }
    pyy /= (ld)members[j].size();
    pzz /= (ld)members[j].size();
    const ld mono[RLBM_NB3] = {e,      px,      py,      pz,      e * e,   e * px, e * py,
                               e * pz, px * px, px * py, px * pz, pyy,     py * pz, pzz};
    for (int a = 0; a < RLBM_NB3; ++a) tab->rowm3d[j][a] = (double)mono[a];
  }
  if (d->precision == RLBM_FP32_DEV) {
    // deviation reference f^ref = f^eq(n_ref, T_ref, u = 0): raw moments of
    // the Maxwell-Juttner distribution at rest (rank <= 3), their centred
    // combinations a^ref, f^ref_j = R_j . a^ref and the moments of f^ref
    const ld nref = d->n_ref > 0 ? d->n_ref : 1.0L, Tref = d->T_ref > 0 ? d->T_ref : 1.0L;
    c.n_ref = (double)nref;
    c.T_ref = (double)Tref;
    const ld e = nref * (3.0L * Tref + m * k1k2_ld(m / Tref)), P = nref * Tref, h = e + P;
    const ld a3 = nref * m * m + 6.0L * Tref * h, b3 = -Tref * h;
    const ld U[4] = {1.0L, 0.0L, 0.0L, 0.0L};
    auto eta = [](int a, int b) { return a != b ? 0.0L : (a == 0 ? 1.0L : -1.0L); };
    ld Mr[RLBM_NO3];
    for (int i = 0; i < RLBM_NO3; ++i) {
      const int a = kO3Idx[i][0], b = kO3Idx[i][1], cc = kO3Idx[i][2];
      if (a < 0)
        Mr[i] = (e - 3.0L * P) / (m * m);
      else if (b < 0)
        Mr[i] = nref * U[a];
      else if (cc < 0)
        Mr[i] = h * U[a] * U[b] - P * eta(a, b);
      else
        Mr[i] = a3 * U[a] * U[b] * U[cc] + b3 * (eta(a, b) * U[cc] + eta(a, cc) * U[b] + eta(b, cc) * U[a]);
    }
    ld aref[RLBM_NO3];
    for (int a = 0; a < RLBM_NO3; ++a) {
      ld sum = 0;
      for (int r = 0; r < RLBM_NO3; ++r) sum += B[a * RLBM_NO3 + r] * Mr[r];
      aref[a] = sum;
      c.o3_aref[a] = (double)sum;
    }
    const O3Act& act = kO3Act[d->dim];
    ld refm[RLBM_NB3] = {};
    for (int j = 0; j < Q; ++j) {
      ld fr = 0;
      for (int r = 0; r < act.n; ++r) fr += (ld)tab->rowo3[j][r] * aref[(int)act.m[r]];
      for (int a = 0; a < RLBM_NB3; ++a) {
        const ld mono = (ld)tab->rowm3d[j][a];
        refm[a] += fr * mono;
        tab->rowm3f[j][a] = (float)mono;
        tab->rowm3f_lo[j][a] = (float)(mono - (ld)tab->rowm3f[j][a]);
      }
      for (int r = 0; r < RLBM_ROWO3; ++r) {
        tab->rowo3f[j][r] = (float)tab->rowo3[j][r];
        tab->rowo3f_lo[j][r] = (float)((ld)tab->rowo3[j][r] - (ld)tab->rowo3f[j][r]);
      }
    }
    for (int a = 0; a < RLBM_NB3; ++a) c.ref_mom3[a] = (double)refm[a];
  }
  return RLBM_OK;
}

int rlbm_build_table(const rlbm_stencil_desc* d, rlbm_stencil_info* info, RlbmTable* tab, char* err,
                     size_t errlen) {
  if (!d || !d->group_base || !(d->zeta > 0) || d->dim < 1 || d->dim > 3 || d->precision < RLBM_FP64 ||
      d->precision > RLBM_FP16_DEV || !(d->order == 0 || d->order == 2 || d->order == 3) ||
      d->n_groups != (d->order == 3 ? 11 : 6)) {
    set_err(err, errlen,
            "invalid stencil description (order 2: 6 groups, order 3: 11 groups; zeta > 0; dim 1|2|3)");
    return RLBM_EINVAL;
  }
  for (int i = 0; i < 3 * d->n_groups; ++i)
    if (d->group_base[i] < 0 || d->group_base[i] > 64) {
      set_err(err, errlen, "group base components must be in [0, 64]");
      return RLBM_EINVAL;
    }
  if (d->order == 3) return build_table_o3(d, info, tab, err, errlen);
  Stencil st((ld)d->zeta, d->n_groups, d->group_base);
  for (int g = 0; g < 6; ++g)
    for (int h = g + 1; h < 6; ++h)
      if (st.orbit[g] == st.orbit[h]) {
        set_err(err, errlen, "repeated velocity group");
        return RLBM_EINVAL;
      }

  ld v0 = d->v0;
  ld wlo = 0, whi = 0;
  if (d->weights && !(v0 > 0)) {
    set_err(err, errlen, "given weights need a given v0");
    return RLBM_EINVAL;
  }
  if (!(v0 > 0)) {
    const int rc = positive_window([&st](ld v) { return st.min_weight(v); }, st.vmax, d, wlo, whi, err, errlen);
    if (rc) return rc;
    v0 = 0.5L * (wlo + whi);
  }
  if (!(v0 < st.vmax)) {
    set_err(err, errlen, "v0 too large: a group would move faster than light");
    return RLBM_EINVAL;
  }
  std::vector<ld> w;
  if (d->weights) {
    for (int g = 0; g < 6; ++g) w.push_back((ld)d->weights[g]);
  } else if (!st.weights(v0, w)) {
    set_err(err, errlen, "singular quadrature system for this group set");
    return RLBM_ENOSTENCIL;
  }
  for (ld x : w)
    if (!(x > 0)) {
      set_err(err, errlen, "quadrature weights not all positive at this v0");
      return RLBM_ENOSTENCIL;
    }

  // populations, orthonormality check over all 14 x 14 pairs
  Basis B((ld)d->zeta);
  std::vector<Pop> pops;
  std::vector<std::array<ld, 4>> mom;
  st.populations(v0, pops, mom);
  ld G[14][14] = {};
  std::vector<std::array<ld, 14>> Jall(pops.size());
  for (size_t i = 0; i < pops.size(); ++i) {
    B.eval14(mom[i].data(), Jall[i].data());
    ld wi = w[pops[i].g];
    for (int l = 0; l < 14; ++l)
      for (int k = 0; k < 14; ++k) G[l][k] += wi * Jall[i][l] * Jall[i][k];
  }
  ld res = 0;
  for (int l = 0; l < 14; ++l)
    for (int k = 0; k < 14; ++k) res = std::max(res, fabsl(G[l][k] - (l == k ? 1.0L : 0.0L)));
  // condition number of the system matrix of the quadrature problem at v0
  // (rows: the pairs l <= k of polynomials, columns: groups, entries
  // sum over the group's populations of J_l J_k): sqrt of the eigenvalue
  // ratio of A^T A
  ld cond = INFINITY;
  {
    std::vector<ld> AtA(36, 0.0L);
    std::vector<ld> row(6);
    for (int l = 0; l < 14; ++l)
      for (int k = l; k < 14; ++k) {
        std::fill(row.begin(), row.end(), 0.0L);
        for (size_t i = 0; i < pops.size(); ++i) row[pops[i].g] += Jall[i][l] * Jall[i][k];
        for (int g = 0; g < 6; ++g)
          for (int h = 0; h < 6; ++h) AtA[g * 6 + h] += row[g] * row[h];
      }
    std::vector<ld> ev;
    jacobi_eigenvalues(6, AtA, ev);
    const ld mx = *std::max_element(ev.begin(), ev.end()), mn = *std::min_element(ev.begin(), ev.end());
    if (mn > 0) cond = sqrtl(mx / mn);
  }
  if (!(res < 1e-10L)) {
    set_err(err, errlen, "orthonormality conditions not satisfied by this group set");
    return RLBM_ENOSTENCIL;
  }

  // classes: (group, nx, ny) in 2D, (group, nx) in 1D; in 3D every
  // population is its own class
  std::map<std::tuple<int, int, int, int>, int> key2class;
  std::vector<std::vector<int>> members;
  for (size_t i = 0; i < pops.size(); ++i) {
    auto key = std::make_tuple(pops[i].g, pops[i].n[0], d->dim >= 2 ? pops[i].n[1] : 0,
                               d->dim == 3 ? pops[i].n[2] : 0);
    auto it = key2class.find(key);
    if (it == key2class.end()) {
      key2class[key] = (int)members.size();
      members.push_back({(int)i});
    } else {
      members[it->second].push_back((int)i);
    }
  }
  int Q = (int)members.size();
  if (Q > RLBM_QMAX) {
    set_err(err, errlen, "stencil has more population classes than the library supports");
    return RLBM_EINVAL;
  }
  int max_shift = 0, sx_max = 0, sy_max = 0, sz_max = 0;
  for (auto& p : pops) {
    sx_max = std::max(sx_max, abs(p.n[0]));
    if (d->dim >= 2) sy_max = std::max(sy_max, abs(p.n[1]));
    if (d->dim == 3) sz_max = std::max(sz_max, abs(p.n[2]));
  }
  max_shift = std::max(sx_max, std::max(sy_max, sz_max));
  if (max_shift > 16) {
    set_err(err, errlen, "displacements above 16 lattice sites are not supported");
    return RLBM_EINVAL;
  }

  if (info) {
    memset(info, 0, sizeof(*info));
    info->q3 = (int)pops.size();
    info->q = Q;
    info->v0 = (double)v0;
    info->v0_lo = (double)wlo;
    info->v0_hi = (double)whi;
    for (int g = 0; g < 6; ++g) info->weights[g] = (double)w[g];
    info->ortho_residual = (double)res;
    info->max_shift = max_shift;
    info->cond = (double)cond;
  }
  if (!tab) return RLBM_OK;

  memset(tab, 0, sizeof(*tab));
  RlbmConsts& c = tab->c;
  c.Q = Q;
  c.order = 2;
  c.dim = d->dim;
  c.precision = d->precision;
  c.max_shift = max_shift;
  c.sx_max = sx_max;
  c.sy_max = sy_max;
  c.sz_max = sz_max;
  c.zeta = d->zeta;
  c.inv_zeta = (double)(1.0L / (ld)d->zeta);
  c.v0 = (double)v0;
  c.a1 = (double)B.a1;
  c.invA = (double)(1.0L / B.A);
  c.invB = (double)(1.0L / B.B);
  c.c1 = (double)B.c1;
  c.c0 = (double)B.c0;
  c.inv_s3C = (double)(1.0L / (sqrtl(3.0L) * B.C));
  c.d0 = (double)B.d0;
  c.invD = (double)(1.0L / B.D);
  c.invE = (double)(1.0L / B.E);

  std::vector<std::array<ld, RLBM_NB>> Mld(Q);
  std::vector<std::array<ld, 3>> pj(Q);
  for (int j = 0; j < Q; ++j) {
    const Pop& p0 = pops[members[j][0]];
    tab->nx[j] = p0.n[0];
    tab->ny[j] = d->dim >= 2 ? p0.n[1] : 0;
    tab->nz[j] = d->dim == 3 ? p0.n[2] : 0;
    const auto& m0 = mom[members[j][0]];
    pj[j] = {m0[0], m0[1], d->dim >= 2 ? m0[2] : 0.0L};
    tab->pz[j] = d->dim == 3 ? (double)m0[3] : 0.0;
    for (int k = 0; k < RLBM_NB; ++k) {
      ld s = 0;
      for (int i : members[j]) s += w[pops[i].g] * Jall[i][kInPlane[k]];
      Mld[j][k] = s;
    }
  }

  // deviation reference: f^ref_j = n_ref sum_k b_k(rest, T_ref) M_jk
  ld nref = d->n_ref > 0 ? d->n_ref : 1.0L;
  ld Tref = d->T_ref > 0 ? d->T_ref : 1.0L;
  c.n_ref = (double)nref;
  c.T_ref = (double)Tref;
  ld zr = (ld)d->zeta / Tref;
  ld R = k1k2_ld(zr);
  ld b[RLBM_NB] = {};
  b[0] = R / (ld)d->zeta;
  b[1] = (1.0L - B.a1 * b[0]) / B.A;
  ld q = (ld)d->zeta * R + 4.0L * Tref;  // mbar K3(z)/K2(z)
  b[4] = (q - Tref + B.c1 + B.c0 * b[0]) / (sqrtl(3.0L) * B.C);
  for (int k = 0; k < RLBM_NB; ++k) c.nb_ref[k] = (double)(nref * b[k]);
  ld refm[9] = {};
  for (int j = 0; j < Q; ++j) {
    ld fr = 0;
    for (int k = 0; k < RLBM_NB; ++k) fr += nref * b[k] * Mld[j][k];
    ld p0 = pj[j][0], px = pj[j][1], py = pj[j][2];
    ld v[9] = {p0, px, py, p0 * p0, p0 * px, p0 * py, px * px, px * py, py * py};
    for (int a = 0; a < 9; ++a) refm[a] += fr * v[a];
    tab->scale[j] = (float)fr;
    tab->inv_scale[j] = (float)(1.0L / fr);
  }
  for (int a = 0; a < 9; ++a) c.ref_mom[a] = (double)refm[a];
  for (int j = 0; j < Q; ++j) {
    tab->dnx[j] = tab->nx[j];
    tab->dny[j] = tab->ny[j];
    tab->fnx[j] = (float)tab->nx[j];
    tab->fny[j] = (float)tab->ny[j];
    tab->p0[j] = (double)pj[j][0];
    tab->px[j] = (double)pj[j][1];
    tab->py[j] = (double)pj[j][2];
    tab->fp0[j] = (float)pj[j][0];
    tab->fpx[j] = (float)pj[j][1];
    tab->fpy[j] = (float)pj[j][2];
    // In the FP16 mode the kernels work on the stored ratios h_j = d_j / f^ref_j,
    // so the float rows carry the class's scale: equilibrium coefficients are
    // divided by f^ref_j and moment monomials multiplied by it.
    const bool ratio = d->precision == RLBM_FP16_DEV;
    const ld fref = ratio ? (ld)tab->scale[j] : 1.0L;
    const bool split = d->precision == RLBM_FP32_DEV;
    for (int k = 0; k < RLBM_NB; ++k) {
      tab->M[k][j] = (double)Mld[j][k];
      tab->Mf[k][j] = (float)Mld[j][k];
      tab->rowf[j][k] = (float)(Mld[j][k] / fref);
      tab->rowd[j][k] = (double)Mld[j][k];
      tab->rowf_lo[j][k] = split ? (float)(Mld[j][k] - (ld)tab->rowf[j][k]) : 0.0f;
    }
    tab->rowf[j][RLBM_R_NX] = tab->fnx[j];
    tab->rowf[j][RLBM_R_NY] = tab->fny[j];
    tab->rowf[j][RLBM_R_INVSCALE] = tab->inv_scale[j];
    tab->rowd[j][RLBM_R_NX] = tab->dnx[j];
    tab->rowd[j][RLBM_R_NY] = tab->dny[j];
    // moment monomials p^a p^b, products taken in long double
    const ld p0 = pj[j][0], px = pj[j][1], py = pj[j][2];
    const ld mono[9] = {p0, px, py, p0 * p0, p0 * px, p0 * py, px * px, px * py, py * py};
    for (int a = 0; a < 9; ++a) {
      tab->rowmf[j][a] = (float)(mono[a] * fref);
      tab->rowmd[j][a] = (double)mono[a];
      tab->rowmf_lo[j][a] = split ? (float)(mono[a] - (ld)tab->rowmf[j][a]) : 0.0f;
    }
    tab->rowmf[j][RLBM_RM_SCALE] = tab->scale[j];
  }
  if (d->dim == 3) {
    // rows of the 3D step kernel: every population is a class of one
    ld rb[RLBM_NB3] = {};
    rb[0] = b[0];
    rb[1] = b[1];
    rb[5] = b[4];
    ld ref3[RLBM_NB3] = {};
    for (int k = 0; k < RLBM_NB3; ++k) c.nb_ref3[k] = (double)(nref * rb[k]);
    const bool ratio = d->precision == RLBM_FP16_DEV;
    const bool split = d->precision == RLBM_FP32_DEV;
    for (int j = 0; j < Q; ++j) {
      const int i = members[j][0];
      const ld wi = w[pops[i].g];
      ld M3[RLBM_NB3];
      ld fr = 0;
      for (int k = 0; k < RLBM_NB3; ++k) {
        M3[k] = wi * Jall[i][k];
        fr += nref * rb[k] * M3[k];
      }
      const ld p0 = mom[i][0], px = mom[i][1], py = mom[i][2], pz = mom[i][3];
      const ld mono[RLBM_NB3] = {p0,      px,      py,      pz,      p0 * p0, p0 * px, p0 * py,
                                 p0 * pz, px * px, px * py, px * pz, py * py, py * pz, pz * pz};
      for (int a = 0; a < RLBM_NB3; ++a) ref3[a] += fr * mono[a];
      const ld fref = ratio ? (ld)(float)fr : 1.0L;
      for (int k = 0; k < RLBM_NB3; ++k) {
        tab->row3d[j][k] = (double)M3[k];
        tab->row3f[j][k] = (float)(M3[k] / fref);
        tab->row3f_lo[j][k] = split ? (float)(M3[k] - (ld)tab->row3f[j][k]) : 0.0f;
      }
      const int nv[3] = {pops[i].n[0], pops[i].n[1], pops[i].n[2]};
      for (int a = 0; a < 3; ++a) {
        tab->row3d[j][RLBM_R3_NX + a] = (double)nv[a];
        tab->row3f[j][RLBM_R3_NX + a] = (float)nv[a];
      }
      tab->row3f[j][RLBM_R3_INVSCALE] = (float)(1.0L / (ld)(float)fr);
      for (int a = 0; a < RLBM_NB3; ++a) {
        tab->rowm3d[j][a] = (double)mono[a];
        tab->rowm3f[j][a] = (float)(mono[a] * fref);
        tab->rowm3f_lo[j][a] = split ? (float)(mono[a] - (ld)tab->rowm3f[j][a]) : 0.0f;
      }
      tab->rowm3f[j][RLBM_RM3_SCALE] = (float)fr;
      tab->scale[j] = (float)fr;
      tab->inv_scale[j] = (float)(1.0L / (ld)(float)fr);
    }
    for (int a = 0; a < RLBM_NB3; ++a) c.ref_mom3[a] = (double)ref3[a];
  }
  return RLBM_OK;
}

uint64_t rlbm_table_fingerprint(const RlbmTable* t) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  const int Q = t->c.Q;
  mix(&t->c.Q, sizeof(int));
  mix(&t->c.dim, sizeof(int));
  mix(&t->c.precision, sizeof(int));
  mix(t->nx, sizeof(int) * Q);
  mix(t->ny, sizeof(int) * Q);
  for (int j = 0; j < Q; ++j) {
    mix(t->rowmf[j], sizeof(float) * 9);
    mix(t->rowf[j], sizeof(float) * RLBM_NB);
    mix(t->rowmf_lo[j], sizeof(float) * 9);
    mix(t->rowf_lo[j], sizeof(float) * RLBM_NB);
  }
  // float64 constants compiled into the generated kernels
  const RlbmConsts& c = t->c;
  const double cs[] = {c.zeta, c.inv_zeta, c.v0, c.a1, c.invA, c.invB, c.c1, c.c0, c.inv_s3C, c.d0, c.invD, c.invE};
  mix(cs, sizeof cs);
  mix(c.ref_mom, sizeof c.ref_mom);
  mix(c.nb_ref, sizeof c.nb_ref);
  if (c.dim == 3) {
    // rows and constants of the 3D step
    mix(t->nz, sizeof(int) * Q);
    for (int j = 0; j < Q; ++j) {
      mix(t->rowm3f[j], sizeof(float) * RLBM_NB3);
      mix(t->rowm3f_lo[j], sizeof(float) * RLBM_NB3);
      mix(t->row3f[j], sizeof(float) * (RLBM_R3_NZ + 1));
      mix(t->row3f_lo[j], sizeof(float) * RLBM_NB3);
    }
    mix(c.ref_mom3, sizeof c.ref_mom3);
    mix(c.nb_ref3, sizeof c.nb_ref3);
  }
  if (c.order == 3) {
    // rows of the third-order step
    mix(t->nz, sizeof(int) * Q);
    for (int j = 0; j < Q; ++j) {
      mix(t->rowm3d[j], sizeof(double) * RLBM_NB3);
      mix(t->rowm3f[j], sizeof(float) * RLBM_NB3);
      mix(t->rowm3f_lo[j], sizeof(float) * RLBM_NB3);
      mix(t->rowo3[j], sizeof(double) * RLBM_ROWO3);
      mix(t->rowo3f[j], sizeof(float) * RLBM_ROWO3);
      mix(t->rowo3f_lo[j], sizeof(float) * RLBM_ROWO3);
    }
  }
  return h;
}

static thread_local char g_err[512];

extern "C" int rlbm_solve_stencil(const rlbm_stencil_desc* desc, rlbm_stencil_info* info) {
  return rlbm_build_table(desc, info, nullptr, g_err, sizeof(g_err));
}

extern "C" int rlbm_class_table(const rlbm_stencil_desc* desc, int cap, int* disp, double* mom, double* M) {
  std::unique_ptr<RlbmTable> holder(new RlbmTable);
  RlbmTable& tab = *holder;
  rlbm_stencil_info info;
  int rc = rlbm_build_table(desc, &info, &tab, g_err, sizeof(g_err));
  if (rc) return rc;
  if (cap < info.q || !disp || !mom || !M) {
    snprintf(g_err, sizeof(g_err), "class table capacity %d < %d", cap, info.q);
    return RLBM_EINVAL;
  }
  for (int j = 0; j < info.q; ++j) {
    disp[2 * j] = tab.nx[j];
    disp[2 * j + 1] = tab.ny[j];
    mom[3 * j] = tab.p0[j];
    mom[3 * j + 1] = tab.px[j];
    mom[3 * j + 2] = tab.py[j];
    for (int k = 0; k < RLBM_NB; ++k) M[RLBM_NB * j + k] = tab.M[k][j];
  }
  return RLBM_OK;
}

// Temperature T(u) solving u + zeta = 3T + zeta K1(zeta/T)/K2(zeta/T)
// (eq. relativistic-eos, T_R = 1) by Newton's method from above (the function
// is convex in T); long double.
static ld eos_temperature_ld(ld u, ld zeta) {
  ld e = u + zeta;
  ld t = std::min(u / 1.5L, e / 3.0L);
  bool done = false;
  for (int it = 0; it < 40; ++it) {
    ld z = zeta / t;
    ld r = k1k2_ld(z);
    ld F = 3 * t + zeta * r - e;
    ld dF = 3 - z * z * r * r - 3 * z * r + z * z;
    ld d = F / dF;
    t -= d;
    if (done) break;
    if (fabsl(d) <= 1e-12L * t) done = true;  // quadratic convergence: one more step
  }
  return t;
}

void rlbm_build_eos_table(double zeta, double (*out)[RLBM_EOS_DEG]) {
  const int D = RLBM_EOS_DEG;
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int o = 0; o < RLBM_EOS_NOCT; ++o) {
    ld base = ldexpl(1.0L, RLBM_EOS_KMIN + o);
    for (int piece = 0; piece < 4; ++piece) {
      ld a = base * (1.0L + 0.25L * piece), b = base * (1.0L + 0.25L * (piece + 1));
      ld g[RLBM_EOS_DEG];
      for (int i = 0; i < D; ++i) {
        ld t = cosl(pi * (i + 0.5L) / D);
        ld u = a + (b - a) * (t + 1.0L) * 0.5L;
        g[i] = eos_temperature_ld(u, (ld)zeta) / u;
      }
      for (int j = 0; j < D; ++j) {
        ld s = 0;
        for (int i = 0; i < D; ++i) s += g[i] * cosl(pi * j * (i + 0.5L) / D);
        s *= 2.0L / D;
        if (j == 0) s *= 0.5L;
        out[o * 4 + piece][j] = (double)s;
      }
    }
  }
}

extern "C" int rlbm_eos_temperature_host(double zeta, const double* e, int n, double* T) {
  if (!(zeta > 0) || !e || !T || n < 0) return RLBM_EINVAL;
  std::unique_ptr<double[][RLBM_EOS_DEG]> tab(new double[RLBM_EOS_NOCT * 4][RLBM_EOS_DEG]);
  rlbm_build_eos_table(zeta, tab.get());
  for (int i = 0; i < n; ++i) {
    double u = e[i] - zeta;
    int ex;
    double m = frexp(u, &ex);
    int o = ex - 1 - RLBM_EOS_KMIN;
    if (!(u > 0) || o < 0 || o >= RLBM_EOS_NOCT) {
      T[i] = (double)eos_temperature_ld((ld)u, (ld)zeta);
      continue;
    }
    double m2 = 2.0 * m;
    int piece = std::min((int)((m2 - 1.0) * 4.0), 3);
    double t = (m2 - 1.0 - 0.25 * piece) * 8.0 - 1.0;
    const double* c = tab[o * 4 + piece];
    double b1 = 0, b2 = 0;
    for (int j = RLBM_EOS_DEG - 1; j >= 1; --j) {
      double b0 = fma(2.0 * t, b1, c[j] - b2);
      b2 = b1;
      b1 = b0;
    }
    T[i] = u * fma(t, b1, c[0] - b2);
  }
  return RLBM_OK;
}

const char* rlbm_global_error() { return g_err; }
void rlbm_set_global_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
