// Build-time generator of the fixed-stencil class code.
//
// For each stencil of the configured workloads it builds the library's own
// class table (the same code the library runs at rlbm_init_stencil) and emits
// straight-line device code for the two class loops of the float32 and
// float16 step kernels, with the table rows as literal constants:
//
//   moments:      m_k += sum_j f_j R_jk        (R: the moment monomials)
//   equilibrium:  f^eq_j = sum_k nb_k M_jk     (M: the equilibrium rows)
//
// The merged in-plane classes of a stencil built from full-symmetric groups
// fall into orbits of the square's symmetry group D4: {(0,0)}, the 4 classes
// (+-a, 0), (0, +-a), the 4 classes (+-a, +-a) and the 8 classes (+-a, +-b),
// (+-b, +-a), each with one energy p^0.  Within an orbit, sums and differences
// of member values (butterflies x + y, x - y) separate the symmetry classes of
// the rows, after which most row coefficients vanish.  For a transform T made
// of butterflies (on member pairs of the fast Walsh-Hadamard stages, each pair
// used or not), R_orbit = T^T C with C = (T^T)^-1 R_orbit, and
//
//   moments:      B = T f_orbit, m_k += C_ok B_o
//   equilibrium:  g = C' nb, f^eq_orbit = T^T g   (butterflies in reverse order)
//
// for the nonzero entries only.  Entries below 1e-12 of the orbit's largest
// row entry are symmetry zeros; every transform is checked to reproduce the
// rows to that accuracy, and the cheapest one (additions plus multiply-adds)
// is chosen, separately for the moments and for the equilibrium.
//
// For float32 storage every coefficient is emitted as a float pair hi + lo
// (hi its nearest float, lo the float nearest to the remainder): the moments
// collect the lo products in nine accumulators of their own, and the lo part
// of the equilibrium is subtracted from f - f^eq before the relaxation.  A
// float coefficient alone would bias every step by its rounding (about 2^-25
// relative), and that bias accumulates in the conserved quantities.
//
// 3D stencils (every population a class of its own) are factored the same
// way over sign orbits: the populations whose displacements differ only in
// the signs of their nonzero components (1, 2, 4 or 8 members, see orbits3).
// The third-order stencil of Fig. 2b (eleven groups at mbar = 7.5) gets the
// same treatment for its 14 moment monomials and its 30 equilibrium rows in
// float64 and float32, emitted as the two passes of the third-order step,
// with the pulls and stores inside each orbit's block (gen_struct_o3).
//
// The output also carries each stencil's table fingerprint; the library uses
// a generated kernel only for a context whose table has the same fingerprint.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "rlbm_stencil.h"

typedef long double ld;

struct Fixed {
  const char* name;
  int base[18];
  double zeta, v0;
};

// The 2D stencils of the configured workloads (group bases of Appendix C,
// mbar, v0 inside each stencil's positive-weight window).
static const Fixed kFixed[] = {
    {"zeta1", {0, 0, 0, 2, 0, 0, 3, 0, 0, 3, 2, 0, 3, 2, 2, 4, 0, 0}, 1.0, 0.2403918860},
    {"zeta5", {0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1, 2, 0, 0, 2, 1, 0}, 5.0, 0.398},
    {"zeta036", {0, 0, 0, 3, 3, 0, 5, 4, 2, 5, 3, 3, 6, 3, 0, 6, 2, 2}, 0.36, 0.1488231854},
    {"zeta10", {0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1, 2, 0, 0, 2, 1, 0}, 10.0, 0.3752119693},
};

// A value of the generated straight-line code: a literal zero, or a named
// variable (possibly negated).
struct Val {
  bool zero = true;
  bool neg = false;
  std::string name;
};

struct Emitter {
  std::string out;
  int tmp = 0;
  std::string type = "float";  // arithmetic type of the emitted temporaries
  void line(const std::string& s) { out += "    " + s + "\n"; }
  std::string fresh(const char* p) { return std::string(p) + std::to_string(tmp++); }
  // a + s b with symbolic zeros
  Val addsub(const Val& a, const Val& b, bool sub) {
    if (b.zero) return a;
    Val nb = b;
    if (sub) nb.neg = !nb.neg;
    if (a.zero) return nb;
    Val r;
    r.zero = false;
    r.name = fresh("t");
    // a.name (sign a) + nb.name (sign nb)
    std::string e;
    if (!a.neg && !nb.neg) e = a.name + " + " + nb.name;
    else if (!a.neg && nb.neg) e = a.name + " - " + nb.name;
    else if (a.neg && !nb.neg) e = nb.name + " - " + a.name;
    else {
      e = a.name + " + " + nb.name;
      r.neg = true;
    }
    line("const " + type + " " + r.name + " = " + e + ";");
    return r;
  }
  // in-place fast Walsh-Hadamard transform (Sylvester order)
  void fwht(std::vector<Val>& v) {
    const int n = (int)v.size();
    for (int h = 1; h < n; h *= 2)
      for (int i = 0; i < n; i += 2 * h)
        for (int j = i; j < i + h; ++j) {
          Val x = v[j], y = v[j + h];
          v[j] = addsub(x, y, false);
          v[j + h] = addsub(x, y, true);
        }
  }
};

// double literal that reads back to the same value
static std::string dlit(double x) {
  char buf[64];
  snprintf(buf, sizeof buf, "%.17e", x);
  return buf;
}

static std::string flit(ld x) {
  char b[64];
  snprintf(b, sizeof b, "%.9ef", (double)(float)x);
  return b;
}

// A coefficient as float: its nearest float (hi) and, when split, the float
// nearest to the remainder (lo), so that hi + lo carries it to about 2^-48.
static ld hi_of(ld x) { return (ld)(float)x; }
static ld lo_of(ld x, bool split) { return split ? (ld)(float)(x - hi_of(x)) : 0.0L; }

// Orbits of the classes: lists of class indices in canonical member order.
static std::vector<std::vector<int>> orbits(const RlbmTable& t) {
  const int Q = t.c.Q;
  std::map<std::tuple<double, int, int>, std::vector<int>> by;
  for (int j = 0; j < Q; ++j) {
    const int ax = abs(t.nx[j]), ay = abs(t.ny[j]);
    by[std::make_tuple(t.p0[j], std::max(ax, ay), std::min(ax, ay))].push_back(j);
  }
  std::vector<std::vector<int>> res;
  for (auto& kv : by) {
    const int a = std::get<1>(kv.first), b = std::get<2>(kv.first);
    std::vector<std::pair<int, int>> want;  // canonical member displacements
    if (a == 0) want = {{0, 0}};
    else if (b == 0) want = {{a, 0}, {-a, 0}, {0, a}, {0, -a}};
    else if (a == b) want = {{a, a}, {-a, a}, {a, -a}, {-a, -a}};
    else want = {{a, b}, {-a, b}, {a, -b}, {-a, -b}, {b, a}, {-b, a}, {b, -a}, {-b, -a}};
    std::vector<int> m;
    for (auto& w : want)
      for (int j : kv.second)
        if (t.nx[j] == w.first && t.ny[j] == w.second) m.push_back(j);
    if (m.size() == want.size() && m.size() == kv.second.size()) {
      res.push_back(m);
    } else {
      for (int j : kv.second) res.push_back({j});  // not a full orbit: one by one
    }
  }
  return res;
}

typedef std::vector<std::pair<int, int>> Bfly;  // butterflies (i, j): (x_i, x_j) <- (x_i + x_j, x_i - x_j)

// Candidate transforms of an n-member orbit: every subset of the pairs of the
// fast Walsh-Hadamard stages (in stage order).
static std::vector<Bfly> candidates(int n) {
  std::vector<std::pair<int, int>> pairs;
  for (int h = 1; h < n; h *= 2)
    for (int i = 0; i < n; i += 2 * h)
      for (int j = i; j < i + h; ++j) pairs.push_back({j, j + h});
  std::vector<Bfly> res;
  const int np = (int)pairs.size();
  for (int mask = 0; mask < (1 << np); ++mask) {
    Bfly b;
    for (int p = 0; p < np; ++p)
      if (mask >> p & 1) b.push_back(pairs[p]);
    res.push_back(b);
  }
  return res;
}

// T (n x n) of a butterfly sequence: B = T x.
static std::vector<std::vector<ld>> tmatrix(int n, const Bfly& b) {
  std::vector<std::vector<ld>> T(n, std::vector<ld>(n, 0));
  for (int i = 0; i < n; ++i) T[i][i] = 1;
  for (auto& p : b)
    for (int c = 0; c < n; ++c) {
      const ld x = T[p.first][c], y = T[p.second][c];
      T[p.first][c] = x + y;
      T[p.second][c] = x - y;
    }
  return T;
}

// C solving T^T C = R (Gaussian elimination with partial pivoting, long
// double), symmetry zeros cleared; false if the result does not reproduce R.
static bool solve_rows(const std::vector<std::vector<ld>>& T, const std::vector<std::vector<ld>>& R,
                       std::vector<std::vector<ld>>& C) {
  const int n = (int)R.size(), K = (int)R[0].size();
  std::vector<std::vector<ld>> A(n, std::vector<ld>(n + K));
  for (int i = 0; i < n; ++i) {
    for (int o = 0; o < n; ++o) A[i][o] = T[o][i];
    for (int k = 0; k < K; ++k) A[i][n + k] = R[i][k];
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
    if (fabsl(A[piv][c]) < 1e-30L) return false;
    std::swap(A[c], A[piv]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const ld f = A[r][c] / A[c][c];
      for (int q = c; q < n + K; ++q) A[r][q] -= f * A[c][q];
    }
  }
  ld mx = 0;
  for (auto& r : R)
    for (ld v : r) mx = std::max(mx, fabsl(v));
  C.assign(n, std::vector<ld>(K, 0));
  for (int o = 0; o < n; ++o)
    for (int k = 0; k < K; ++k) {
      const ld v = A[o][n + k] / A[o][o];
      C[o][k] = fabsl(v) <= 1e-12L * mx ? 0 : v;
    }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < K; ++k) {
      ld s = 0;
      for (int o = 0; o < n; ++o) s += T[o][i] * C[o][k];
      if (fabsl(s - R[i][k]) > 1e-12L * (mx > 0 ? mx : 1)) return false;
    }
  return true;
}

static int nnz(const std::vector<ld>& r) {
  int c = 0;
  for (ld v : r) c += v != 0;
  return c;
}

// Operations of the equilibrium side: row products of g, then the reversed
// butterflies on g with symbolic zeros.
static int eq_cost(const std::vector<std::vector<ld>>& C, const Bfly& b) {
  const int n = (int)C.size();
  int ops = 0;
  std::vector<bool> nz(n);
  for (int o = 0; o < n; ++o) {
    const int k = nnz(C[o]);
    nz[o] = k > 0;
    ops += k;
  }
  for (int i = (int)b.size() - 1; i >= 0; --i) {
    const int x = b[i].first, y = b[i].second;
    if (nz[x] && nz[y]) ops += 2;
    nz[x] = nz[y] = nz[x] || nz[y];
  }
  return ops;
}

struct OrbitPlan {
  std::vector<int> members;
  Bfly bm, be;                           // transforms of the moment and equilibrium sides
  std::vector<std::vector<ld>> Cm, Ce;   // coefficients
};

// Rows of the class loops: for float32 storage the float rows plus their
// rounding remainders (the row values to about 2^-48), otherwise the float
// rows as they are.
static OrbitPlan plan_rows(const std::vector<int>& o, const std::vector<std::vector<ld>>& Rm,
                           const std::vector<std::vector<ld>>& Re) {
  const int n = (int)o.size();
  OrbitPlan pl;
  pl.members = o;
  int best_m = 1 << 30, best_e = 1 << 30;
  for (const Bfly& b : candidates(n)) {
    const auto T = tmatrix(n, b);
    std::vector<std::vector<ld>> C;
    if (solve_rows(T, Rm, C)) {
      int cost = 2 * (int)b.size();
      for (auto& r : C) cost += nnz(r);
      if (cost < best_m) {
        best_m = cost;
        pl.bm = b;
        pl.Cm = C;
      }
    }
    if (solve_rows(T, Re, C)) {
      const int cost = eq_cost(C, b);
      if (cost < best_e) {
        best_e = cost;
        pl.be = b;
        pl.Ce = C;
      }
    }
  }
  return pl;
}

static OrbitPlan plan_orbit(const RlbmTable& t, const std::vector<int>& o) {
  std::vector<std::vector<ld>> Rm, Re;
  for (int j : o) {
    std::vector<ld> rm(9), re(RLBM_NB);
    for (int k = 0; k < 9; ++k) rm[k] = (ld)t.rowmf[j][k] + (ld)t.rowmf_lo[j][k];
    for (int k = 0; k < RLBM_NB; ++k) re[k] = (ld)t.rowf[j][k] + (ld)t.rowf_lo[j][k];
    Rm.push_back(rm);
    Re.push_back(re);
  }
  return plan_rows(o, Rm, Re);
}

static std::string gen_struct(const char* sname, const RlbmTable& t) {
  const int Q = t.c.Q;
  const bool split = t.c.precision == RLBM_FP32_DEV;
  std::vector<OrbitPlan> plans;
  for (auto& o : orbits(t)) plans.push_back(plan_orbit(t, o));
  Emitter em;
  std::string s;
  s += "struct " + std::string(sname) + " {\n";
  s += "  static constexpr int Q = " + std::to_string(Q) + ";\n";
  s += "  static constexpr int orbits = " + std::to_string(plans.size()) + ";\n";
  // class displacements (lattice units), indexed by template constants only
  std::string sx = "  static constexpr int kNx[" + std::to_string(Q) + "] = {";
  std::string sy = "  static constexpr int kNy[" + std::to_string(Q) + "] = {";
  for (int j = 0; j < Q; ++j) {
    sx += (j ? ", " : "") + std::to_string(t.nx[j]);
    sy += (j ? ", " : "") + std::to_string(t.ny[j]);
  }
  s += sx + "};\n" + sy + "};\n";
  // moments
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of class " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    std::vector<Val> v(n);
    for (int i = 0; i < n; ++i) {
      v[i].zero = false;
      v[i].name = "f[" + std::to_string(pl.members[i]) + "]";
    }
    for (auto& p : pl.bm) {
      const Val x = v[p.first], y = v[p.second];
      v[p.first] = em.addsub(x, y, false);
      v[p.second] = em.addsub(x, y, true);
    }
    for (int o = 0; o < n; ++o)
      for (int k = 0; k < 9; ++k) {
        if (pl.Cm[o][k] == 0 || v[o].zero) continue;
        const ld c = v[o].neg ? -pl.Cm[o][k] : pl.Cm[o][k];
        em.line("m[" + std::to_string(k) + "] = fmaf(" + v[o].name + ", " + flit(hi_of(c)) + ", m[" +
                std::to_string(k) + "]);");
        const ld cl = lo_of(c, split);
        if (cl != 0)
          em.line("ml[" + std::to_string(k) + "] = fmaf(" + v[o].name + ", " + flit(cl) + ", ml[" +
                  std::to_string(k) + "]);");
      }
    em.line("}");
  }
  s += "  static __device__ __forceinline__ void moments(const float (&f)[" + std::to_string(Q) +
       "], float (&m)[9], float (&ml)[9]) {\n" + em.out + "  }\n";
  // equilibrium, relaxation and stores, one orbit at a time
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of class " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    // g = C' nb for the float parts of the coefficients and, when split,
    // gl for their remainders; the same butterflies take both to the classes
    auto chain = [&](bool lo, std::vector<Val>& g) {
      for (int o = 0; o < n; ++o) {
        std::string e;
        for (int k = 0; k < RLBM_NB; ++k) {
          if (pl.Ce[o][k] == 0) continue;
          const ld c = lo ? lo_of(pl.Ce[o][k], split) : hi_of(pl.Ce[o][k]);
          if (c == 0) continue;
          if (e.empty()) e = "nb[" + std::to_string(k) + "] * " + flit(c);
          else e = "fmaf(nb[" + std::to_string(k) + "], " + flit(c) + ", " + e + ")";
        }
        if (e.empty()) continue;
        g[o].zero = false;
        g[o].name = em.fresh(lo ? "gl" : "g");
        em.line("const float " + g[o].name + " = " + e + ";");
      }
      for (int i = (int)pl.be.size() - 1; i >= 0; --i) {
        const int x = pl.be[i].first, y = pl.be[i].second;
        const Val a = g[x], b = g[y];
        g[x] = em.addsub(a, b, false);
        g[y] = em.addsub(a, b, true);
      }
    };
    std::vector<Val> g(n), gl(n);
    chain(false, g);
    chain(true, gl);
    auto ref = [](const Val& v) { return v.zero ? std::string("0.0f") : (v.neg ? "(-" + v.name + ")" : v.name); };
    for (int i = 0; i < n; ++i) {
      const int j = pl.members[i];
      std::string om = "W0";
      if (t.ny[j] != 0) om = "fmaf(WY, " + flit((ld)t.ny[j]) + ", " + om + ")";
      if (t.nx[j] != 0) om = "fmaf(WX, " + flit((ld)t.nx[j]) + ", " + om + ")";
      const std::string fj = "f[" + std::to_string(j) + "]";
      // f - f^eq is small next to f, so subtracting the remainder part there
      // keeps it (a correction below half an ulp of f would be lost in f)
      std::string diff = fj + " - " + ref(g[i]);
      if (!gl[i].zero) diff = "(" + diff + ") - " + ref(gl[i]);
      em.line(fj + " = fmaf(-(" + om + "), " + diff + ", " + fj + ");");
      em.line("st.template put<" + std::to_string(j) + ">(" + fj + ");");
    }
    em.line("}");
  }
  s += "  template <class Store>\n  static __device__ __forceinline__ void collide(float (&f)[" + std::to_string(Q) +
       "], const float (&nb)[RLBM_NB], float W0, float WX, float WY, Store& st) {\n" + em.out + "  }\n";
  // the stencil's float64 constants (Appendix A at mbar, deviation reference)
  const RlbmConsts& c = t.c;
  s += "  struct C {\n";
  const std::pair<const char*, double> sc[] = {{"zeta", c.zeta}, {"inv_zeta", c.inv_zeta}, {"v0", c.v0},
                                                {"a1", c.a1},     {"invA", c.invA},         {"invB", c.invB},
                                                {"c1", c.c1},     {"c0", c.c0},             {"inv_s3C", c.inv_s3C},
                                                {"d0", c.d0},     {"invD", c.invD},         {"invE", c.invE}};
  for (auto& kv : sc) s += "    static constexpr double " + std::string(kv.first) + " = " + dlit(kv.second) + ";\n";
  auto table_fn = [&s](const char* name, const double* v, int n) {
    s += "    static __device__ __forceinline__ constexpr double " + std::string(name) + "(int k) {\n";
    s += "      switch (k) {\n";
    for (int k = 0; k < n; ++k) s += "        case " + std::to_string(k) + ": return " + dlit(v[k]) + ";\n";
    s += "      }\n      return 0.0;\n    }\n";
  };
  table_fn("ref_mom", c.ref_mom, 9);
  table_fn("nb_ref", c.nb_ref, RLBM_NB);
  s += "  };\n";
  s += "};\n";
  return s;
}

// 3D stencils: every population is a class of its own.  Populations that
// differ only in the signs of their displacement components form sign orbits
// of 1, 2, 4 or 8 members (one energy p^0), taken in the order of the sign
// bits of their nonzero components (x first), so that the butterflies of the
// Walsh-Hadamard stages pair members that differ in one sign.
static std::vector<std::vector<int>> orbits3(const RlbmTable& t) {
  const int Q = t.c.Q;
  std::map<std::tuple<double, int, int, int>, std::vector<int>> by;
  for (int j = 0; j < Q; ++j)
    by[std::make_tuple(t.p0[j], abs(t.nx[j]), abs(t.ny[j]), abs(t.nz[j]))].push_back(j);
  std::vector<std::vector<int>> res;
  for (auto& kv : by) {
    const int a[3] = {std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first)};
    int axes[3], k = 0;
    for (int d = 0; d < 3; ++d)
      if (a[d]) axes[k++] = d;
    std::vector<int> m;
    for (int sbits = 0; sbits < (1 << k); ++sbits) {
      int want[3] = {a[0], a[1], a[2]};
      for (int i = 0; i < k; ++i)
        if (sbits >> i & 1) want[axes[i]] = -want[axes[i]];
      for (int j : kv.second)
        if (t.nx[j] == want[0] && t.ny[j] == want[1] && t.nz[j] == want[2]) m.push_back(j);
    }
    if ((int)m.size() == (1 << k) && m.size() == kv.second.size()) {
      res.push_back(m);
    } else {
      for (int j : kv.second) res.push_back({j});  // not a full sign orbit: one by one
    }
  }
  return res;
}

static std::string gen_struct3(const char* sname, const RlbmTable& t) {
  const int Q = t.c.Q;
  const bool split = t.c.precision == RLBM_FP32_DEV;
  std::vector<OrbitPlan> plans;
  for (auto& o : orbits3(t)) {
    std::vector<std::vector<ld>> Rm, Re;
    for (int j : o) {
      std::vector<ld> rm(RLBM_NB3), re(RLBM_NB3);
      for (int k = 0; k < RLBM_NB3; ++k) rm[k] = (ld)t.rowm3f[j][k] + (ld)t.rowm3f_lo[j][k];
      for (int k = 0; k < RLBM_NB3; ++k) re[k] = (ld)t.row3f[j][k] + (ld)t.row3f_lo[j][k];
      Rm.push_back(rm);
      Re.push_back(re);
    }
    plans.push_back(plan_rows(o, Rm, Re));
  }
  Emitter em;
  std::string s;
  s += "struct " + std::string(sname) + " {\n";
  s += "  static constexpr int Q = " + std::to_string(Q) + ";\n";
  s += "  static constexpr int orbits = " + std::to_string(plans.size()) + ";\n";
  const std::string nb3 = std::to_string(RLBM_NB3);
  // moments
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of population " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    std::vector<Val> v(n);
    for (int i = 0; i < n; ++i) {
      v[i].zero = false;
      v[i].name = "f[" + std::to_string(pl.members[i]) + "]";
    }
    for (auto& q : pl.bm) {
      const Val x = v[q.first], y = v[q.second];
      v[q.first] = em.addsub(x, y, false);
      v[q.second] = em.addsub(x, y, true);
    }
    for (int o = 0; o < n; ++o)
      for (int k = 0; k < RLBM_NB3; ++k) {
        if (pl.Cm[o][k] == 0 || v[o].zero) continue;
        const ld c = v[o].neg ? -pl.Cm[o][k] : pl.Cm[o][k];
        em.line("m[" + std::to_string(k) + "] = fmaf(" + v[o].name + ", " + flit(hi_of(c)) + ", m[" +
                std::to_string(k) + "]);");
        const ld cl = lo_of(c, split);
        if (cl != 0)
          em.line("ml[" + std::to_string(k) + "] = fmaf(" + v[o].name + ", " + flit(cl) + ", ml[" +
                  std::to_string(k) + "]);");
      }
    em.line("}");
  }
  s += "  static __device__ __forceinline__ void moments(const float (&f)[" + std::to_string(Q) + "], float (&m)[" +
       nb3 + "], float (&ml)[" + nb3 + "]) {\n" + em.out + "  }\n";
  // equilibrium, relaxation and stores, one orbit at a time
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of population " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    auto chain = [&](bool lo, std::vector<Val>& g) {
      for (int o = 0; o < n; ++o) {
        std::string e;
        for (int k = 0; k < RLBM_NB3; ++k) {
          if (pl.Ce[o][k] == 0) continue;
          const ld c = lo ? lo_of(pl.Ce[o][k], split) : hi_of(pl.Ce[o][k]);
          if (c == 0) continue;
          if (e.empty()) e = "nb[" + std::to_string(k) + "] * " + flit(c);
          else e = "fmaf(nb[" + std::to_string(k) + "], " + flit(c) + ", " + e + ")";
        }
        if (e.empty()) continue;
        g[o].zero = false;
        g[o].name = em.fresh(lo ? "gl" : "g");
        em.line("const float " + g[o].name + " = " + e + ";");
      }
      for (int i = (int)pl.be.size() - 1; i >= 0; --i) {
        const int x = pl.be[i].first, y = pl.be[i].second;
        const Val a = g[x], b = g[y];
        g[x] = em.addsub(a, b, false);
        g[y] = em.addsub(a, b, true);
      }
    };
    std::vector<Val> g(n), gl(n);
    chain(false, g);
    chain(true, gl);
    auto ref = [](const Val& v) { return v.zero ? std::string("0.0f") : (v.neg ? "(-" + v.name + ")" : v.name); };
    for (int i = 0; i < n; ++i) {
      const int j = pl.members[i];
      std::string om = "W0";
      if (t.nz[j] != 0) om = "fmaf(WZ, " + flit((ld)t.nz[j]) + ", " + om + ")";
      if (t.ny[j] != 0) om = "fmaf(WY, " + flit((ld)t.ny[j]) + ", " + om + ")";
      if (t.nx[j] != 0) om = "fmaf(WX, " + flit((ld)t.nx[j]) + ", " + om + ")";
      const std::string fj = "f[" + std::to_string(j) + "]";
      std::string diff = fj + " - " + ref(g[i]);
      if (!gl[i].zero) diff = "(" + diff + ") - " + ref(gl[i]);
      em.line(fj + " = fmaf(-(" + om + "), " + diff + ", " + fj + ");");
      em.line("st.template put<" + std::to_string(j) + ">(" + fj + ");");
    }
    em.line("}");
  }
  s += "  template <class Store>\n  static __device__ __forceinline__ void collide(float (&f)[" + std::to_string(Q) +
       "], const float (&nb)[" + nb3 + "], float W0, float WX, float WY, float WZ, Store& st) {\n" + em.out +
       "  }\n";
  s += "};\n";
  return s;
}

// Third order (Sec. III.A, III.D): the two passes of the third-order step
// for one stencil, orbit by orbit.  Pass 1 pulls an orbit's populations and
// adds their 14 moment monomials (the ones that can be nonzero on a lattice
// of this dimension); pass 2 pulls them again, forms their equilibria from
// the 30 projections on the centred monomials (the active ones, in the
// table's packed order), relaxes and stores.  Float64 storage takes double
// coefficients; float32 deviation storage hi/lo float pairs as above.
static std::string dlit_any(ld x, bool dbl) { return dbl ? dlit((double)x) : flit(x); }

static std::string gen_struct_o3(const char* sname, const RlbmTable& t) {
  const int Q = t.c.Q, dim = t.c.dim;
  const bool dbl = t.c.precision == RLBM_FP64;
  const bool split = t.c.precision == RLBM_FP32_DEV;
  const O3Act& act = kO3Act[dim];
  std::vector<OrbitPlan> plans;
  for (auto& o : (dim == 3 ? orbits3(t) : orbits(t))) {
    std::vector<std::vector<ld>> Rm, Re;
    for (int j : o) {
      std::vector<ld> rm(RLBM_NB3, 0), re(act.n);
      for (int k = 0; k < RLBM_NB3; ++k)
        if (o3_mom_active(dim, k))
          rm[k] = dbl ? (ld)t.rowm3d[j][k] : (ld)t.rowm3f[j][k] + (ld)t.rowm3f_lo[j][k];
      for (int k = 0; k < act.n; ++k) re[k] = dbl ? (ld)t.rowo3[j][k] : (ld)t.rowo3f[j][k] + (ld)t.rowo3f_lo[j][k];
      Rm.push_back(rm);
      Re.push_back(re);
    }
    plans.push_back(plan_rows(o, Rm, Re));
  }
  const std::string A = dbl ? "double" : "float";
  const std::string fma = dbl ? "fma" : "fmaf";
  auto hi = [&](ld c) { return dbl ? c : hi_of(c); };
  auto lo = [&](ld c) { return dbl ? 0.0L : lo_of(c, split); };
  Emitter em;
  em.type = A;
  std::string s;
  s += "struct " + std::string(sname) + " {\n";
  s += "  static constexpr int Q = " + std::to_string(Q) + ";\n";
  s += "  static constexpr int orbits = " + std::to_string(plans.size()) + ";\n";
  // pass 1
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of class " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    std::vector<Val> v(n);
    for (int i = 0; i < n; ++i) {
      v[i].zero = false;
      v[i].name = "f" + std::to_string(pl.members[i]);
      em.line("const " + A + " " + v[i].name + " = pl.template get<" + std::to_string(pl.members[i]) + ">();");
    }
    for (auto& q : pl.bm) {
      const Val x = v[q.first], y = v[q.second];
      v[q.first] = em.addsub(x, y, false);
      v[q.second] = em.addsub(x, y, true);
    }
    for (int o = 0; o < n; ++o)
      for (int k = 0; k < RLBM_NB3; ++k) {
        if (pl.Cm[o][k] == 0 || v[o].zero) continue;
        const ld c = v[o].neg ? -pl.Cm[o][k] : pl.Cm[o][k];
        em.line("m[" + std::to_string(k) + "] = " + fma + "(" + v[o].name + ", " + dlit_any(hi(c), dbl) + ", m[" +
                std::to_string(k) + "]);");
        const ld cl = lo(c);
        if (cl != 0)
          em.line("ml[" + std::to_string(k) + "] = fmaf(" + v[o].name + ", " + flit(cl) + ", ml[" +
                  std::to_string(k) + "]);");
      }
    em.line("}");
    em.line("__builtin_amdgcn_sched_barrier(0);");
  }
  s += "  template <class Pull>\n  static __device__ __forceinline__ void moments(Pull& pl, " + A + " (&m)[" +
       std::to_string(RLBM_NB3) + "], " + A + " (&ml)[" + std::to_string(RLBM_NB3) + "]) {\n" + em.out + "  }\n";
  // pass 2
  em.out.clear();
  for (auto& pl : plans) {
    const int n = (int)pl.members.size();
    em.line("{  // orbit of class " + std::to_string(pl.members[0]) + " (" + std::to_string(n) + ")");
    for (int i = 0; i < n; ++i)
      em.line("const " + A + " f" + std::to_string(pl.members[i]) + " = pl.template get<" +
              std::to_string(pl.members[i]) + ">();");
    auto chain = [&](bool low, std::vector<Val>& g) {
      for (int o = 0; o < n; ++o) {
        std::string e;
        for (int k = 0; k < act.n; ++k) {
          if (pl.Ce[o][k] == 0) continue;
          const ld c = low ? lo(pl.Ce[o][k]) : hi(pl.Ce[o][k]);
          if (c == 0) continue;
          const std::string mk = "M[" + std::to_string((int)act.m[k]) + "]";
          if (e.empty()) e = mk + " * " + dlit_any(c, dbl);
          else e = fma + "(" + mk + ", " + dlit_any(c, dbl) + ", " + e + ")";
        }
        if (e.empty()) continue;
        g[o].zero = false;
        g[o].name = em.fresh(low ? "gl" : "g");
        em.line("const " + A + " " + g[o].name + " = " + e + ";");
      }
      for (int i = (int)pl.be.size() - 1; i >= 0; --i) {
        const int x = pl.be[i].first, y = pl.be[i].second;
        const Val a = g[x], b = g[y];
        g[x] = em.addsub(a, b, false);
        g[y] = em.addsub(a, b, true);
      }
    };
    std::vector<Val> g(n), gl(n);
    chain(false, g);
    if (split) chain(true, gl);
    const std::string zero = dbl ? "0.0" : "0.0f";
    auto ref = [&](const Val& v) { return v.zero ? zero : (v.neg ? "(-" + v.name + ")" : v.name); };
    for (int i = 0; i < n; ++i) {
      const int j = pl.members[i];
      std::string om = "W0";
      if (t.nz[j] != 0) om = fma + "(WZ, " + dlit_any((ld)t.nz[j], dbl) + ", " + om + ")";
      if (t.ny[j] != 0) om = fma + "(WY, " + dlit_any((ld)t.ny[j], dbl) + ", " + om + ")";
      if (t.nx[j] != 0) om = fma + "(WX, " + dlit_any((ld)t.nx[j], dbl) + ", " + om + ")";
      const std::string fj = "f" + std::to_string(j);
      std::string diff = fj + " - " + ref(g[i]);
      if (split && !gl[i].zero) diff = "(" + diff + ") - " + ref(gl[i]);
      em.line("st.template put<" + std::to_string(j) + ">(" + fma + "(-(" + om + "), " + diff + ", " + fj + "));");
    }
    em.line("}");
    em.line("__builtin_amdgcn_sched_barrier(0);");
  }
  s += "  template <class Pull, class Store>\n  static __device__ __forceinline__ void collide(Pull& pl, const " + A +
       " (&M)[" + std::to_string(RLBM_NO3) + "], " + A + " W0, " + A + " WX, " + A + " WY, " + A + " WZ, Store& st) {\n" +
       em.out + "  }\n";
  s += "};\n";
  return s;
}

// The third-order stencil of Fig. 2b (groups G1, G2, G3, G4, G5, G8, G9,
// G10, G12, G13, G15) at mbar = 7.5 with the library's own v0 (middle of the
// positive-weight window), for 2D (merged classes) and 3D lattices.
static const int kFig2b[33] = {0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1, 2, 0, 0, 2, 1, 1, 2, 2, 1,
                               2, 2, 2, 3, 1, 0, 3, 2, 0, 3, 1, 1};

// The 3D stencils of the configured workloads (G1..G6 at mbar = 5 and the
// mbar = 1 stencil), at the v0 the workloads use.
static const Fixed kFixed3[] = {
    {"zeta5", {0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1, 2, 0, 0, 2, 1, 0}, 5.0, 0.398},
    {"zeta1", {0, 0, 0, 2, 0, 0, 3, 0, 0, 3, 2, 0, 3, 2, 2, 4, 0, 0}, 1.0, 0.2403918860},
};

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s output.h\n", argv[0]);
    return 2;
  }
  std::string out;
  out += "// Generated at build time by gen_fixed_stencils.cpp from the library's own\n";
  out += "// class tables: straight-line class loops of the configured 2D and 3D stencils.\n";
  out += "#pragma once\n#include <stdint.h>\n\nnamespace rlbm_fixed {\n\n";
  std::string table = "static const struct { const char* name; int precision; uint64_t fingerprint; } kFixedTables[] = {\n";
  int id = 0;
  std::string dispatch;
  for (const Fixed& f : kFixed) {
    for (int prec : {RLBM_FP32_DEV, RLBM_FP16_DEV}) {
      rlbm_stencil_desc d;
      memset(&d, 0, sizeof d);
      d.dim = 2;
      d.n_groups = 6;
      d.group_base = f.base;
      d.zeta = f.zeta;
      d.v0 = f.v0;
      d.precision = prec;
      std::unique_ptr<RlbmTable> t(new RlbmTable);
      rlbm_stencil_info info;
      char err[512];
      if (rlbm_build_table(&d, &info, t.get(), err, sizeof err) != RLBM_OK) {
        fprintf(stderr, "%s: %s\n", f.name, err);
        return 1;
      }
      char sname[64];
      snprintf(sname, sizeof sname, "S%d", id);
      out += "// " + std::string(f.name) + (prec == RLBM_FP32_DEV ? ", float32" : ", float16") + " storage\n";
      out += gen_struct(sname, *t);
      out += "\n";
      char row[256];
      snprintf(row, sizeof row, "    {\"%s\", %d, 0x%016llxull},\n", f.name, prec,
               (unsigned long long)rlbm_table_fingerprint(t.get()));
      table += row;
      dispatch += " X(" + std::to_string(id) + ", " + sname + ", " + std::to_string(prec) + ")";
      ++id;
    }
  }
  table += "};\nconstexpr int kNumFixed = " + std::to_string(id) + ";\n";
  table += "// X(id, struct, precision) for every generated kernel\n#define RLBM_FIXED_KERNELS(X)" + dispatch + "\n";
  // 3D stencils: moments and collision of every population
  std::string table3 = "static const struct { const char* name; int precision; uint64_t fingerprint; } kFixed3Tables[] = {\n";
  std::string dispatch3;
  int id3 = 0;
  for (const Fixed& f : kFixed3) {
    for (int prec : {RLBM_FP32_DEV, RLBM_FP16_DEV}) {
      rlbm_stencil_desc d;
      memset(&d, 0, sizeof d);
      d.dim = 3;
      d.n_groups = 6;
      d.group_base = f.base;
      d.zeta = f.zeta;
      d.v0 = f.v0;
      d.precision = prec;
      std::unique_ptr<RlbmTable> t(new RlbmTable);
      rlbm_stencil_info info;
      char err[512];
      if (rlbm_build_table(&d, &info, t.get(), err, sizeof err) != RLBM_OK) {
        fprintf(stderr, "%s (3D): %s\n", f.name, err);
        return 1;
      }
      char sname[64];
      snprintf(sname, sizeof sname, "T%d", id3);
      out += "// " + std::string(f.name) + " 3D" + (prec == RLBM_FP32_DEV ? ", float32" : ", float16") + " storage\n";
      out += gen_struct3(sname, *t);
      out += "\n";
      char row[256];
      snprintf(row, sizeof row, "    {\"%s\", %d, 0x%016llxull},\n", f.name, prec,
               (unsigned long long)rlbm_table_fingerprint(t.get()));
      table3 += row;
      dispatch3 += " X(" + std::to_string(id3) + ", " + sname + ", " + std::to_string(prec) + ")";
      ++id3;
    }
  }
  // third order: the Fig. 2b stencil at mbar = 7.5
  std::string tableo3 =
      "static const struct { const char* name; int precision; int dim; uint64_t fingerprint; } kFixedO3Tables[] = {\n";
  std::string dispatcho3;
  int ido3 = 0;
  const int o3cases[4][2] = {{2, RLBM_FP64}, {2, RLBM_FP32_DEV}, {3, RLBM_FP32_DEV}, {3, RLBM_FP64}};
  for (const auto& oc : o3cases) {
    {
      const int dim = oc[0], prec = oc[1];
      rlbm_stencil_desc d;
      memset(&d, 0, sizeof d);
      d.dim = dim;
      d.order = 3;
      d.n_groups = 11;
      d.group_base = kFig2b;
      d.zeta = 7.5;
      d.v0 = 0.0;
      d.precision = prec;
      std::unique_ptr<RlbmTable> t(new RlbmTable);
      rlbm_stencil_info info;
      char err[512];
      if (rlbm_build_table(&d, &info, t.get(), err, sizeof err) != RLBM_OK) {
        fprintf(stderr, "third order (%dD): %s\n", dim, err);
        return 1;
      }
      char sname[64];
      snprintf(sname, sizeof sname, "U%d", ido3);
      out += "// third order, Fig. 2b stencil, " + std::to_string(dim) + "D" +
             (prec == RLBM_FP64 ? ", float64" : ", float32") + " storage\n";
      out += gen_struct_o3(sname, *t);
      out += "\n";
      char row[256];
      snprintf(row, sizeof row, "    {\"fig2b\", %d, %d, 0x%016llxull},\n", prec, dim,
               (unsigned long long)rlbm_table_fingerprint(t.get()));
      tableo3 += row;
      dispatcho3 += " X(" + std::to_string(ido3) + ", " + sname + ", " + std::to_string(prec) + ", " +
                    std::to_string(dim) + ")";
      ++ido3;
    }
  }
  tableo3 += "};\nconstexpr int kNumFixedO3 = " + std::to_string(ido3) + ";\n";
  tableo3 += "// X(id, struct, precision, dim) for every generated third-order kernel\n#define RLBM_FIXEDO3_KERNELS(X)" +
             dispatcho3 + "\n";
  table3 += "};\nconstexpr int kNumFixed3 = " + std::to_string(id3) + ";\n";
  table3 += "// X(id, struct, precision) for every generated 3D kernel\n#define RLBM_FIXED3_KERNELS(X)" + dispatch3 + "\n";
  out += table + "\n" + table3 + "\n" + tableo3 + "\n}  // namespace rlbm_fixed\n";
  FILE* fp = fopen(argv[1], "w");
  if (!fp) {
    perror(argv[1]);
    return 1;
  }
  fputs(out.c_str(), fp);
  fclose(fp);
  return 0;
}
