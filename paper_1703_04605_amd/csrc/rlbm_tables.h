// Shared host/device layout of the per-stencil constant table and the kernel
// argument blocks of the relativistic lattice Boltzmann library.
#pragma once
#include <stdint.h>

#define RLBM_QMAX 160   // population classes per stencil (6 groups: <= 150)
#define RLBM_NB 10      // second-order polynomials that survive U_z = 0

// Polynomial order of the 10 in-plane coefficients (Appendix A labels):
//   0: J^(0)     1: J^(1)_0   2: J^(1)_x   3: J^(1)_y   4: J^(2)_00
//   5: J^(2)_0x  6: J^(2)_0y  7: J^(2)_xx  8: J^(2)_yy  9: J^(2)_xy
// where Appendix A's J_xx is (p_y^2 - p_z^2)/(2E) and its J_yy is
// (-2 p_x^2 + p_y^2 + p_z^2)/(2 sqrt(3) E).

struct RlbmConsts {
  int Q;          // population classes (planes)
  int dim;        // 1 or 2
  int precision;  // RLBM_FP64 / RLBM_FP32_DEV / RLBM_FP16_DEV
  int max_shift;
  double zeta;    // mbar = m / T_R
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
};

// Per-block health / statistics slot, accumulated by the step kernel.
struct RlbmSlot {
  uint32_t flags;
  uint32_t iter_max;
  uint64_t iter_sum;
};

struct RlbmStepArgs {
  const void* src;
  void* dst;
  long long plane;     // elements per population plane
  int nx, ny;
  int bc_x, bc_y;      // RLBM_BC_*
  int shift;           // 1: pull f_j(x - n_j) (post-collision state), 0: read f_j(x)
  int x_small, y_small;  // lattice side <= max shift: use modular wrap
  int blocks_x;        // blocks per row
  int tau_mode;
  double tau;          // constant tau
  double tk1, tk2;     // eta/s: tau = 1/2 + tk1 (4 - ln(tk2 n / T^3)) / T
  double landau_tol;
  int landau_maxit;
  const RlbmTable* tab;
  RlbmSlot* slots;     // one per block (logical index)
};

struct RlbmMomArgs {
  const void* src;
  long long plane;
  int nx, ny, bc_x, bc_y, shift, x_small, y_small;
  double landau_tol;
  int landau_maxit;
  const RlbmTable* tab;
  double *n, *eps, *T, *P, *ux, *uy, *raw9;
};

struct RlbmInitArgs {
  void* dst;
  long long plane;
  int nx, ny;
  const double *n, *T, *ux, *uy;
  const RlbmTable* tab;
};
