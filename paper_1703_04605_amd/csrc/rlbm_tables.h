// Shared host/device layout of the per-stencil constant table and the kernel
// argument blocks of the relativistic lattice Boltzmann library.
#pragma once
#include <stdint.h>

#define RLBM_QMAX 192   // population classes per stencil (6 groups: <= 150; 11 groups: more)
#define RLBM_NB 10      // second-order polynomials that survive U_z = 0

// Inverse equation of state T(u), u = eps/n - mbar (kinetic energy per
// particle): T/u as a Chebyshev series on each quarter of each octave
// 2^k <= u < 2^(k+1), k = RLBM_EOS_KMIN .. RLBM_EOS_KMIN + RLBM_EOS_NOCT - 1.
#define RLBM_EOS_KMIN (-24)
#define RLBM_EOS_NOCT 48
#define RLBM_EOS_DEG 14

// equilibrium rows: M_j0 .. M_j9, n_x, n_y [, 1/scale] (padded: one wide load)
#define RLBM_ROWF 16
#define RLBM_ROWD 12
enum { RLBM_R_NX = 10, RLBM_R_NY = 11, RLBM_R_INVSCALE = 12 };
// moment rows: p0, px, py, p0 p0, p0 px, p0 py, px px, px py, py py [, scale]
#define RLBM_ROWMF 12
#define RLBM_ROWMD 10
#define RLBM_RM_SCALE 9

// 3D lattices: all 14 second-order polynomials (Appendix A order 0, 1_0,
// 1_x, 1_y, 1_z, 2_00, 2_0x, 2_0y, 2_0z, 2_xx, 2_yy, 2_xz, 2_yz, 2_xy);
// equilibrium rows [M_j0 .. M_j13, n_x, n_y, n_z, 1/scale, 0, 0], moment rows
// [p0, px, py, pz, p0p0, p0px, p0py, p0pz, pxpx, pxpy, pxpz, pypy, pypz,
// pzpz, scale, 0].  Row lengths keep every row a multiple of 16 bytes (the
// kernels read a row as one 16-byte aligned struct).
#define RLBM_NB3 14
#define RLBM_ROW3 20
#define RLBM_ROWM3 16
enum { RLBM_R3_NX = 14, RLBM_R3_NY = 15, RLBM_R3_NZ = 16, RLBM_R3_INVSCALE = 17 };
#define RLBM_RM3_SCALE 14

// Third-order model (Sec. III.A: 30 polynomials of degree <= 3, float64
// only).  With M_m = int f^eq p^{i1} .. p^{ir} d^3p/p^0 (a component of a
// Maxwell-Juttner moment tensor of rank r <= 3, density included) for the 30
// monomials listed in kO3Idx, and q_m the centred, scaled monomials
// ((p0 - c)/s0)^k0 (p_x/sp)^kx (p_y/sp)^ky (p_z/sp)^kz of the same
// exponents, the equilibrium of population j is sum_m R_jm a_m with
// a_m = int f^eq q_m d^3p/p^0 (a binomial combination of the M's) and the
// row R_j built on the host in the q basis (well conditioned at every mbar).
// Rows: [R_j0 .. R_j29, n_x, n_y, n_z, 0].
#define RLBM_NO3 30
#define RLBM_ROWO3 34
enum { RLBM_RO3_NX = 30, RLBM_RO3_NY = 31, RLBM_RO3_NZ = 32 };
// index lists (0 = time component, 1..3 = x, y, z; -1 = unused) of the 30
// monomials: degree 0, 1, 2 and 3, p_z at most once (on the mass shell the
// monomials with p_z^2 or p_z^3 depend on these)
static constexpr signed char kO3Idx[RLBM_NO3][3] = {
    {-1, -1, -1},                                                                     // 1
    {0, -1, -1}, {1, -1, -1}, {2, -1, -1}, {3, -1, -1},                               // p^a
    {0, 0, -1}, {0, 1, -1}, {0, 2, -1}, {0, 3, -1}, {1, 1, -1}, {1, 2, -1},           // p^a p^b
    {1, 3, -1}, {2, 2, -1}, {2, 3, -1},
    {0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 0, 3}, {0, 1, 1}, {0, 1, 2}, {0, 1, 3},      // p^a p^b p^c
    {0, 2, 2}, {0, 2, 3}, {1, 1, 1}, {1, 1, 2}, {1, 1, 3}, {1, 2, 2}, {1, 2, 3},
    {2, 2, 2}, {2, 2, 3}};

// exponent of axis `ax` (0 = time) in monomial m
constexpr int o3_exp(int m, int ax) {
  int e = 0;
  for (int r = 0; r < 3; ++r) e += kO3Idx[m][r] == ax ? 1 : 0;
  return e;
}
// kO3Raw.r[m][k]: index of the monomial p0^k times the spatial part of
// monomial m (k <= o3_exp(m, 0)), -1 beyond
struct O3Raw {
  signed char r[RLBM_NO3][4];
};
constexpr O3Raw make_o3_raw() {
  O3Raw t{};
  for (int m = 0; m < RLBM_NO3; ++m)
    for (int k = 0; k < 4; ++k) {
      t.r[m][k] = -1;
      if (k > o3_exp(m, 0)) continue;
      for (int q = 0; q < RLBM_NO3; ++q)
        if (o3_exp(q, 0) == k && o3_exp(q, 1) == o3_exp(m, 1) && o3_exp(q, 2) == o3_exp(m, 2) &&
            o3_exp(q, 3) == o3_exp(m, 3))
          t.r[m][k] = (signed char)q;
    }
  return t;
}
static constexpr O3Raw kO3Raw = make_o3_raw();

// Monomials whose moments can be nonzero on a lattice of dimension dim (the
// flow has no velocity along the merged axes: in 2D the terms odd in p_z
// vanish, in 1D also those odd in p_y); rows of 1D and 2D classes hold only
// these coefficients, in kO3Idx order, at the front of the row.
constexpr bool o3_active(int dim, int m) {
  return dim == 3 || (o3_exp(m, 3) == 0 && (dim == 2 || o3_exp(m, 2) % 2 == 0));
}
struct O3Act {
  signed char m[RLBM_NO3];
  int n;
};
constexpr O3Act make_o3_act(int dim) {
  O3Act t{};
  t.n = 0;
  for (int m = 0; m < RLBM_NO3; ++m)
    if (o3_active(dim, m)) t.m[t.n++] = (signed char)m;
  return t;
}
static constexpr O3Act kO3Act[4] = {O3Act{}, make_o3_act(1), make_o3_act(2), make_o3_act(3)};
// moments (3D moment-row order) that can be nonzero on a lattice of dimension dim
constexpr bool o3_mom_active(int dim, int k) {
  // 0 N0, 1 Nx, 2 Ny, 3 Nz, 4 T00, 5 T0x, 6 T0y, 7 T0z, 8 Txx, 9 Txy, 10 Txz, 11 Tyy, 12 Tyz, 13 Tzz
  return dim == 3 || (dim == 2 ? (k != 3 && k != 7 && k != 10 && k != 12 && k != 13)
                               : (k == 0 || k == 1 || k == 4 || k == 5 || k == 8));
}

#define RLBM_LANDAU_NEWTON 0      // Newton on det(lambda I - T eta) from lambda = T^00
#define RLBM_LANDAU_FIXED_POINT 1 // eps = T^00 - T^0i u_i, u_i = (T^0i - T^ij u_j)/eps

// Polynomial order of the 10 in-plane coefficients (Appendix A labels):
//   0: J^(0)     1: J^(1)_0   2: J^(1)_x   3: J^(1)_y   4: J^(2)_00
//   5: J^(2)_0x  6: J^(2)_0y  7: J^(2)_xx  8: J^(2)_yy  9: J^(2)_xy
// where Appendix A's J_xx is (p_y^2 - p_z^2)/(2E) and its J_yy is
// (-2 p_x^2 + p_y^2 + p_z^2)/(2 sqrt(3) E).

struct RlbmConsts {
  int Q;          // population classes (planes)
  int order;      // 2 or 3 (equilibrium expansion order)
  int dim;        // 1, 2 or 3
  int precision;  // RLBM_FP64 / RLBM_FP32_DEV / RLBM_FP16_DEV
  int max_shift;
  int sx_max, sy_max, sz_max;  // max |n_x|, max |n_y|, max |n_z| over the classes
  double zeta;    // mbar = m / T_R
  double inv_zeta;
  double v0;
  // Appendix A constants at mbar (T_R = 1):
  double a1;      // mbar K2/K1        (J^(1)_0 offset)
  double invA, invB;
  double c1, c0;  // J^(2)_00 = (p0^2 + c1 p0 + c0) / (sqrt(3) C)
  double inv_s3C;
  double d0;      // mbar K3/K2        (J^(2)_0i offset)
  double invD, invE;
  // deviation reference f^ref = f^eq(n_ref, T_ref, u = 0)
  double n_ref, T_ref;
  double nb_ref[RLBM_NB];  // n_ref * b_k(rest, T_ref)
  double ref_mom[9];       // sum_j f^ref_j (p0, px, py, p0p0, p0px, p0py, pxpx, pxpy, pypy)
  double nb_ref3[RLBM_NB3];  // 3D: n_ref * b_k(rest, T_ref) for all 14 polynomials
  double ref_mom3[RLBM_NB3]; // 3D: sum_j f^ref_j times the 14 monomials of the 3D moment rows
  double o3_c, o3_is0, o3_isp;  // third order: centre c of p0, 1/s0, 1/sp of the q basis
  double o3_aref[RLBM_NO3];     // third order, float32 storage: projections a_m of f^ref
};

struct RlbmTable {
  RlbmConsts c;
  int nx[RLBM_QMAX], ny[RLBM_QMAX];
  double dnx[RLBM_QMAX], dny[RLBM_QMAX];
  double p0[RLBM_QMAX], px[RLBM_QMAX], py[RLBM_QMAX];
  double M[RLBM_NB][RLBM_QMAX];
  float fnx[RLBM_QMAX], fny[RLBM_QMAX];
  float fp0[RLBM_QMAX], fpx[RLBM_QMAX], fpy[RLBM_QMAX];
  float Mf[RLBM_NB][RLBM_QMAX];
  float scale[RLBM_QMAX], inv_scale[RLBM_QMAX];  // FP16: d_j = scale_j * h_j
  double eos[RLBM_EOS_NOCT * 4][RLBM_EOS_DEG];     // inverse EOS pieces
  // Per-class equilibrium rows read by the step kernel with wide scalar loads:
  // [M_j0 .. M_j9, n_x, n_y, 1/scale, 0, 0, 0] (float) and
  // [M_j0 .. M_j9, n_x, n_y] (double).
  float rowf[RLBM_QMAX][RLBM_ROWF] __attribute__((aligned(64)));
  double rowd[RLBM_QMAX][RLBM_ROWD] __attribute__((aligned(64)));
  // Per-class moment rows: the nine monomials p^a p^b of eq.
  // mj-discrete-second-moment (and the FP16 scale), one wide scalar load each.
  float rowmf[RLBM_QMAX][RLBM_ROWMF] __attribute__((aligned(64)));
  double rowmd[RLBM_QMAX][RLBM_ROWMD] __attribute__((aligned(64)));
  // float32 storage: the rounding remainders of the float rows (row value -
  // float row, rounded to float), so that hi + lo carries each coefficient to
  // about 2^-48.  A float row alone biases every step's moments and
  // equilibrium by its rounding (about 2^-25 relative), which accumulates in
  // the conserved quantities over long runs.  Zero in the other modes.
  float rowf_lo[RLBM_QMAX][RLBM_ROWF] __attribute__((aligned(64)));
  float rowmf_lo[RLBM_QMAX][RLBM_ROWMF] __attribute__((aligned(64)));
  // 3D lattices (every population its own class): z displacement, p^z, and
  // the rows of the 3D step kernel (layouts above); float rows carry the
  // FP16 scale as in 2D, and the float32 remainders as in 2D.
  int nz[RLBM_QMAX];
  double pz[RLBM_QMAX];
  double row3d[RLBM_QMAX][RLBM_ROW3] __attribute__((aligned(64)));
  float row3f[RLBM_QMAX][RLBM_ROW3] __attribute__((aligned(64)));
  float row3f_lo[RLBM_QMAX][RLBM_ROW3] __attribute__((aligned(64)));
  double rowm3d[RLBM_QMAX][RLBM_ROWM3] __attribute__((aligned(64)));
  float rowm3f[RLBM_QMAX][RLBM_ROWM3] __attribute__((aligned(64)));
  float rowm3f_lo[RLBM_QMAX][RLBM_ROWM3] __attribute__((aligned(64)));
  // Per-lattice byte offsets of every class from the lowest element a tile
  // can reach (class 0 at (x0 - Sx, y - Sy)): [0, QMAX) in place (the own
  // storage the step writes), [QMAX, 2 QMAX) pulled.  Written on the device
  // by rlbm_init_fields for the lattice in use.
  unsigned offs[2 * RLBM_QMAX] __attribute__((aligned(64)));
  // third-order equilibrium rows (layout above; classes of dim 1 and 2 carry
  // the sums over their members and n_z = 0)
  double rowo3[RLBM_QMAX][RLBM_ROWO3] __attribute__((aligned(64)));
  // float32 storage: the same rows rounded to float, and their rounding
  // remainders (hi + lo carries each coefficient to about 2^-48)
  float rowo3f[RLBM_QMAX][RLBM_ROWO3] __attribute__((aligned(64)));
  float rowo3f_lo[RLBM_QMAX][RLBM_ROWO3] __attribute__((aligned(64)));
};

// Per-block health / statistics slot, accumulated by the step kernel.
struct RlbmSlot {
  uint32_t flags;
  uint32_t iter_max;
  uint64_t iter_sum;
};

// Population storage, row-interleaved: (ny + 2 GY) storage rows, each holding
// the Q class rows of W elements of one lattice row back to back, so f_j at
// site (x, y) lives at j cs + (y + GY) rs + x + GX with cs = W and rs = Q W.
// All classes of a lattice row then share a few hundred KB, and a tile's
// pulls and stores stay within a few pages.  The ghost columns [-Sx, 0),
// [nx, nx+Sx) and rows [-Sy, 0), [ny, ny+Sy) hold copies written by the owner
// sites under the boundary rule, so pulls f_j(x - n_j) need no wrap or clamp.
// 3D lattices stack (nz + 2 GZ) such planes of storage rows, zs elements
// apart (2D: nz = 1, GZ = Sz = 0).
struct RlbmLayout {
  long long cs;     // elements between classes at one site (W)
  long long rs;     // elements between storage rows (Q W)
  long long zs;     // elements between storage planes ((ny + 2 GY) rs)
  long long total;  // elements of the whole buffer (padded)
  int W, GX, GY, GZ;
  int nx, ny, nz;
  int Sx, Sy, Sz;   // ghost widths actually used (max shifts)
  int bc_x, bc_y, bc_z;
};

struct RlbmStepArgs {
  const void* src;
  void* dst;
  RlbmLayout L;
  // Per class, byte offsets from the tile's lowest reachable element (class 0
  // at (x0 - Sx, y - Sy)): offs = source of f_j (j cs + Sy rs + Sx, minus
  // n_y rs + n_x when pulling), offs_st = own storage of f_j; QMAX entries each.
  const unsigned* offs;
  const unsigned* offs_st;
  // The same offsets as arithmetic, for kernels that know n_j at compile
  // time: own_j = fo_base + j fo_cs, source = own_j - n_y fo_rs - n_x fo_es
  // (fo_rs = fo_es = 0 when reading in place).
  unsigned fo_base, fo_cs;
  int fo_rs, fo_es;
  int shift;           // 1: pull f_j(x - n_j) (post-collision state), 0: read f_j(x)
  int tiles_x;         // wave tiles (64 sites) per row
  int ntiles;          // wave tiles of the lattice
  int tau_mode;
  double tau;          // constant tau
  double inv_tau;      // 1 / tau
  double tk1, tk2;     // eta/s: tau = 1/2 + tk1 (4 - ln(tk2 n / T^3)) / T
  double landau_tol;
  int landau_maxit;
  int landau_method;   // RLBM_LANDAU_*
  const RlbmTable* tab;
  RlbmSlot* slots;     // one per block (logical index)
  // warm start: (eps, u_x, u_y) planes of nx ny floats, or nullptr
  float* warm;
  long long warm_plane;
  // learned Landau guess (kernels with the guess only)
  const unsigned short* mlp_frag;
  const float* mlp_bias;
  float mlp_norm[24];  // mx[9], 1/sx[9], my[3], sy[3]
};

struct RlbmMomArgs {
  const void* src;
  RlbmLayout L;
  int shift;
  double landau_tol;
  int landau_maxit;
  int landau_method;
  const RlbmTable* tab;
  double *n, *eps, *T, *P, *ux, *uy, *raw9;
};

struct RlbmInitArgs {
  void* dst;
  RlbmLayout L;
  const double *n, *T, *ux, *uy;
  const RlbmTable* tab;
};
