// Build-time generator of the fixed-stencil class kernels.
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
// (+-b, +-a), each with one energy p^0.  With the orbit's members ordered so
// that the bits of a member's index are its x sign, y sign and x<->y swap,
// the Sylvester-Hadamard matrix H (H H = n I) block-diagonalises the rows:
// R_orbit = H C with C = H R_orbit / n sparse (symmetry zeros).  So
//
//   moments:      B = H f_orbit (fast Walsh-Hadamard transform), m_k += C_ok B_o
//   equilibrium:  g = C' nb, f^eq_orbit = H g
//
// for the nonzero entries only.  Entries whose magnitude is below 1e-12 of the
// orbit's rows are symmetry zeros; the generator checks that H C reproduces
// the rows to that accuracy and otherwise treats the orbit's classes one by one.
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
    line("const float " + r.name + " = " + e + ";");
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

static std::string flit(ld x) {
  char b[64];
  snprintf(b, sizeof b, "%.9ef", (double)(float)x);
  return b;
}

static void hadamard(int n, std::vector<std::vector<int>>& H) {
  H.assign(n, std::vector<int>(n, 1));
  for (int h = 1; h < n; h *= 2)
    for (int i = 0; i < h; ++i)
      for (int j = 0; j < h; ++j) {
        H[i][j + h] = H[i][j];
        H[i + h][j] = H[i][j];
        H[i + h][j + h] = -H[i][j];
      }
}

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

// C = H R / n for the orbit; returns false if H C does not reproduce R.
static bool factor(const std::vector<std::vector<ld>>& R, std::vector<std::vector<ld>>& C) {
  const int n = (int)R.size(), K = (int)R[0].size();
  std::vector<std::vector<int>> H;
  hadamard(n, H);
  ld mx = 0;
  for (auto& r : R)
    for (ld v : r) mx = std::max(mx, fabsl(v));
  C.assign(n, std::vector<ld>(K, 0));
  for (int o = 0; o < n; ++o)
    for (int k = 0; k < K; ++k) {
      ld s = 0;
      for (int i = 0; i < n; ++i) s += H[o][i] * R[i][k];
      s /= n;
      C[o][k] = fabsl(s) <= 1e-12L * mx ? 0 : s;
    }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < K; ++k) {
      ld s = 0;
      for (int o = 0; o < n; ++o) s += H[o][i] * C[o][k];
      if (fabsl(s - R[i][k]) > 1e-12L * (mx > 0 ? mx : 1)) return false;
    }
  return true;
}

static std::string gen_struct(const char* sname, const RlbmTable& t) {
  const int Q = t.c.Q;
  const auto orb0 = orbits(t);
  // orbits that factor; others split into single classes
  std::vector<std::vector<int>> orb;
  for (auto& o : orb0) {
    std::vector<std::vector<ld>> Rm, Re, Cm, Ce;
    for (int j : o) {
      std::vector<ld> rm(9), re(RLBM_NB);
      for (int k = 0; k < 9; ++k) rm[k] = t.rowmf[j][k];
      for (int k = 0; k < RLBM_NB; ++k) re[k] = t.rowf[j][k];
      Rm.push_back(rm);
      Re.push_back(re);
    }
    if (factor(Rm, Cm) && factor(Re, Ce)) orb.push_back(o);
    else
      for (int j : o) orb.push_back({j});
  }
  Emitter em;
  std::string s;
  s += "struct " + std::string(sname) + " {\n";
  s += "  static constexpr int Q = " + std::to_string(Q) + ";\n";
  s += "  static constexpr int orbits = " + std::to_string(orb.size()) + ";\n";
  // moments
  em.out.clear();
  for (auto& o : orb) {
    const int n = (int)o.size();
    std::vector<std::vector<ld>> R, C;
    for (int j : o) {
      std::vector<ld> r(9);
      for (int k = 0; k < 9; ++k) r[k] = t.rowmf[j][k];
      R.push_back(r);
    }
    factor(R, C);
    em.line("{  // orbit of class " + std::to_string(o[0]) + " (" + std::to_string(n) + ")");
    std::vector<Val> v(n);
    for (int i = 0; i < n; ++i) {
      v[i].zero = false;
      v[i].name = "f[" + std::to_string(o[i]) + "]";
    }
    em.fwht(v);
    for (int oo = 0; oo < n; ++oo)
      for (int k = 0; k < 9; ++k) {
        if (C[oo][k] == 0 || v[oo].zero) continue;
        const ld c = v[oo].neg ? -C[oo][k] : C[oo][k];
        em.line("m[" + std::to_string(k) + "] = fmaf(" + v[oo].name + ", " + flit(c) + ", m[" + std::to_string(k) +
                "]);");
      }
    em.line("}");
  }
  s += "  static __device__ __forceinline__ void moments(const float (&f)[" + std::to_string(Q) +
       "], float (&m)[9]) {\n" + em.out + "  }\n";
  // equilibrium, relaxation and stores, one orbit at a time
  em.out.clear();
  for (auto& o : orb) {
    const int n = (int)o.size();
    std::vector<std::vector<ld>> R, C;
    for (int j : o) {
      std::vector<ld> r(RLBM_NB);
      for (int k = 0; k < RLBM_NB; ++k) r[k] = t.rowf[j][k];
      R.push_back(r);
    }
    factor(R, C);
    em.line("{  // orbit of class " + std::to_string(o[0]) + " (" + std::to_string(n) + ")");
    std::vector<Val> g(n);
    for (int oo = 0; oo < n; ++oo) {
      std::string e;
      for (int k = 0; k < RLBM_NB; ++k) {
        if (C[oo][k] == 0) continue;
        if (e.empty()) e = "nb[" + std::to_string(k) + "] * " + flit(C[oo][k]);
        else e = "fmaf(nb[" + std::to_string(k) + "], " + flit(C[oo][k]) + ", " + e + ")";
      }
      if (e.empty()) continue;
      g[oo].zero = false;
      g[oo].name = em.fresh("g");
      em.line("const float " + g[oo].name + " = " + e + ";");
    }
    em.fwht(g);
    for (int i = 0; i < n; ++i) {
      const int j = o[i];
      std::string feq = g[i].zero ? "0.0f" : (g[i].neg ? "(-" + g[i].name + ")" : g[i].name);
      std::string om = "W0";
      if (t.ny[j] != 0) om = "fmaf(WY, " + flit((ld)t.ny[j]) + ", " + om + ")";
      if (t.nx[j] != 0) om = "fmaf(WX, " + flit((ld)t.nx[j]) + ", " + om + ")";
      const std::string fj = "f[" + std::to_string(j) + "]";
      em.line(fj + " = fmaf(-(" + om + "), " + fj + " - " + feq + ", " + fj + ");");
      em.line("st.template put<" + std::to_string(j) + ">(" + fj + ");");
    }
    em.line("}");
  }
  s += "  template <class Store>\n  static __device__ __forceinline__ void collide(float (&f)[" + std::to_string(Q) +
       "], const float (&nb)[RLBM_NB], float W0, float WX, float WY, Store& st) {\n" + em.out + "  }\n";
  s += "};\n";
  return s;
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s output.h\n", argv[0]);
    return 2;
  }
  std::string out;
  out += "// Generated at build time by gen_fixed_stencils.cpp from the library's own\n";
  out += "// class tables: straight-line class loops of the configured 2D stencils.\n";
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
  out += table + "\n}  // namespace rlbm_fixed\n";
  FILE* fp = fopen(argv[1], "w");
  if (!fp) {
    perror(argv[1]);
    return 1;
  }
  fputs(out.c_str(), fp);
  fclose(fp);
  return 0;
}
