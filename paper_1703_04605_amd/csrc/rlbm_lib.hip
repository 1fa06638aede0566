// HIP kernels (gfx950) and C ABI of the relativistic lattice Boltzmann library
// (arXiv:1703.04605, second-order model of Sec. III).
//
// Data layout in HBM: row-interleaved classes, f[y][j][x] with x fastest
// (the Q class rows of one lattice row are consecutive), padded to 128
// elements; two buffers (ping-pong).
// A time step is one fused kernel: each thread owns one site, pulls the Q
// class values f_j(x - n_j) from the previous post-collision state (exact
// streaming, Sec. III.B), keeps them in registers, reduces the nine in-plane
// moments, solves the Landau frame, inverts the equation of state, builds the
// equilibrium from the projections and relaxes (Anderson-Witting), and writes
// the post-collision values to the other buffer.  Each population value is
// read once and written once per step, which is the HBM roofline of the step.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <type_traits>
#include <utility>
#include <cmath>
#include <vector>

#include "../../include/rlbm.h"
#include "rlbm_device.h"
#include "rlbm_mlp.h"
#include "rlbm_stencil.h"
#include "rlbm_tables.h"
#include "rlbm_fixed_stencils.h"  // generated at build time

namespace rlbm {

constexpr int kBlock = 256;
// Step kernel workgroups are single waves: a finished wave frees its slot for
// the next tile at once instead of waiting for the rest of its workgroup.
constexpr int kStepBlock = 64;
constexpr int kWave = 64;
// fourth word of a raw buffer descriptor on CDNA: 32-bit data format, no
// swizzle, untyped loads and stores address bytes
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kRecAll = 0x7FFFFFFF;        // records of a step descriptor
constexpr int kRecOut = (int)0x80000000u;  // a lane offset beyond them
typedef unsigned U32x2 __attribute__((ext_vector_type(2)));
constexpr long long kPlaneAlign = 128;  // elements
constexpr double kHbarC = 0.1973269804; // GeV fm

template <int P> struct Traits;
template <> struct Traits<RLBM_FP64> { using S = double; using A = double; };
template <> struct Traits<RLBM_FP32_DEV> { using S = float; using A = float; };
template <> struct Traits<RLBM_FP16_DEV> { using S = _Float16; using A = float; };

template <int P>
__device__ __forceinline__ typename Traits<P>::A to_arith(typename Traits<P>::S v, TabPtr tb, int j) {
  if constexpr (P == RLBM_FP16_DEV) return (float)v * tb->scale[j];
  else return v;
}

template <int P>
__device__ __forceinline__ typename Traits<P>::S to_store(typename Traits<P>::A v, TabPtr tb, int j) {
  if constexpr (P == RLBM_FP16_DEV) return (_Float16)(v * tb->inv_scale[j]);
  else return v;
}

// Reduces health flags and Landau iteration counts over the wave into the
// wave's own slot (one slot per wave of the persistent grid: no atomics, no
// races).
// Reduction over the 64 lanes of a wave (all active) for a commutative,
// associative op with identity 0: within each row of 16 lanes by DPP lane
// permutations (quad swaps, then rotations by 4 and 8), then over the four
// rows' first lanes.
template <class Op>
__device__ __forceinline__ unsigned wave_reduce(unsigned v, Op op) {
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));  // row_ror:4
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));  // row_ror:8
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return op(op(r0, r1), op(r2, r3));
}

__device__ __forceinline__ void wave_stats(RlbmSlot* slots, int gw, unsigned flags, unsigned iters_max,
                                           unsigned iters_sum) {
  // (a wave's iteration sum, at most 64 (maxit + 1), fits 32 bits)
  const unsigned fl = wave_reduce(flags, [](unsigned a, unsigned b) { return a | b; });
  const unsigned mx = wave_reduce(iters_max, [](unsigned a, unsigned b) { return max(a, b); });
  const unsigned long long sm = wave_reduce(iters_sum, [](unsigned a, unsigned b) { return a + b; });
  if ((threadIdx.x & 63) == 0) {
    RlbmSlot s = slots[gw];
    s.flags |= fl;
    s.iter_max = max(s.iter_max, mx);
    s.iter_sum += sm;
    slots[gw] = s;
  }
}

// Macroscopic state of one site from its moments (float64).
struct Macro {
  double n, eps, T, P, ux, uy, gamma, R;
  int iters;
  unsigned flags;
};

// Newton stopping threshold for a requested tolerance (the last step is taken
// after the step falls below it: quadratic convergence)
__device__ __forceinline__ double newton_thresh(double tol) { return 0.1 * sqrt(tol); }

// guess (eps0, ux0, uy0): starting point of the Landau solve; eps0 <= 0 means
// none (Newton from T^00, fixed point from u = 0)
// (zeta = mbar and its inverse passed in, so that kernels with the stencil's
// constants compiled in need no table read for them)
__device__ __forceinline__ Macro macroscopic_z(TabPtr tb, double zeta, double inv_zeta, double N0, double Nx,
                                               double Ny, double T00, double T0x, double T0y, double Txx,
                                               double Txy, double Tyy, double tol, int maxit, int method,
                                               double eps0, double ux0, double uy0) {
  Macro m;
  m.flags = 0;
  const bool guess = eps0 > 0.0 && eps0 < T00 && ux0 * ux0 + uy0 * uy0 < 1.0;
  m.ux = guess ? ux0 : 0.0;
  m.uy = guess ? uy0 : 0.0;
  if (method == RLBM_LANDAU_NEWTON)
    m.iters = landau_newton(T00, T0x, T0y, Txx, Txy, Tyy, newton_thresh(tol), maxit, m.eps, m.ux, m.uy,
                            guess ? eps0 : T00);
  else
    m.iters = landau_solve(T00, T0x, T0y, Txx, Txy, Tyy, tol, maxit, m.eps, m.ux, m.uy);
  if (m.iters > maxit) m.flags |= RLBM_H_LANDAU;
  const double u2 = m.ux * m.ux + m.uy * m.uy;
  if (!(u2 < 1.0)) m.flags |= RLBM_H_SUPERLUMINAL;
  m.gamma = rsqrt_nr(1.0 - u2);
  m.n = m.gamma * (N0 - m.ux * Nx - m.uy * Ny);
  if (!(m.n > 0.0) || !(m.eps > 0.0)) m.flags |= RLBM_H_RANGE;
  const double e = div_nr(m.eps, m.n);
  m.T = eos_temperature_tab(tb, e, zeta, m.flags);
  m.P = m.n * m.T;
  // K1/K2 at z = zeta/T from the EOS itself: zeta R = e - 3T
  m.R = (e - 3.0 * m.T) * inv_zeta;
  if (!isfinite(m.T) || !isfinite(m.eps) || !isfinite(m.n) || !isfinite(m.R)) m.flags |= RLBM_H_NAN;
  return m;
}

__device__ __forceinline__ Macro macroscopic(TabPtr tb, double N0, double Nx, double Ny,
                                             double T00, double T0x, double T0y, double Txx, double Txy,
                                             double Tyy, double tol, int maxit, int method, double eps0 = 0.0,
                                             double ux0 = 0.0, double uy0 = 0.0) {
  return macroscopic_z(tb, tb->c.zeta, tb->c.inv_zeta, N0, Nx, Ny, T00, T0x, T0y, Txx, Txy, Tyy, tol, maxit,
                       method, eps0, ux0, uy0);
}

// Per-stencil constants of the step: from the table, or compiled in for the
// generated stencils (struct C of rlbm_fixed_stencils.h, same values).
template <class Fx>
struct StepConsts {
  static __device__ __forceinline__ double zeta(TabPtr) { return Fx::C::zeta; }
  static __device__ __forceinline__ double inv_zeta(TabPtr) { return Fx::C::inv_zeta; }
  static __device__ __forceinline__ double v0(TabPtr) { return Fx::C::v0; }
  static __device__ __forceinline__ double ref_mom(TabPtr, int k) { return Fx::C::ref_mom(k); }
  static __device__ __forceinline__ double nb_ref(TabPtr, int k) { return Fx::C::nb_ref(k); }
  static __device__ __forceinline__ ProjConsts proj(TabPtr) {
    using C = typename Fx::C;
    return ProjConsts{C::zeta, C::inv_zeta, C::a1, C::invA, C::invB, C::c1, C::c0, C::inv_s3C, C::d0, C::invD,
                      C::invE};
  }
};
template <>
struct StepConsts<void> {
  static __device__ __forceinline__ double zeta(TabPtr tb) { return tb->c.zeta; }
  static __device__ __forceinline__ double inv_zeta(TabPtr tb) { return tb->c.inv_zeta; }
  static __device__ __forceinline__ double v0(TabPtr tb) { return tb->c.v0; }
  static __device__ __forceinline__ double ref_mom(TabPtr tb, int k) { return tb->c.ref_mom[k]; }
  static __device__ __forceinline__ double nb_ref(TabPtr tb, int k) { return tb->c.nb_ref[k]; }
  static __device__ __forceinline__ ProjConsts proj(TabPtr tb) { return proj_consts(tb); }
};

// ------------------------------------------------------------------ layout

// Ghost cells of one axis: bit i stands for ghost coordinate c_i = i - S
// (i < S) or n + i - S (i >= S); it is set when the boundary rule maps c_i to
// the owner coordinate x (periodic: c mod n; outflow: clamp to [0, n)).
__device__ __forceinline__ unsigned ghost_mask(int x, int n, int S, int bc) {
  unsigned m = 0;
  for (int i = 0; i < 2 * S; ++i) {
    const int c = i < S ? i - S : n + (i - S);
    int src;
    if (bc == RLBM_BC_PERIODIC) {
      // one wrap when n >= S; lattices smaller than the stencil's reach take
      // the remainder
      src = c < 0 ? c + n : (c >= n ? c - n : c);
      if (src < 0 || src >= n) src = ((c % n) + n) % n;
    } else {
      src = min(max(c, 0), n - 1);
    }
    if (src == x) m |= 1u << i;
  }
  return m;
}

__device__ __forceinline__ int ghost_coord(int i, int n, int S) { return i < S ? i - S : n + (i - S); }

// Writes v to every ghost copy of site (x, y) in class q (the owner copy is
// written by the caller).
template <typename S>
__device__ __forceinline__ void store_ghosts(S* __restrict__ q, const RlbmLayout& L, int x, int y, unsigned xm,
                                             unsigned ym, S v) {
  for (unsigned m = xm; m; m &= m - 1)
    q[(long long)(y + L.GY) * L.rs + ghost_coord(__builtin_ctz(m), L.nx, L.Sx) + L.GX] = v;
  for (unsigned r = ym; r; r &= r - 1) {
    const long long row = (long long)(ghost_coord(__builtin_ctz(r), L.ny, L.Sy) + L.GY) * L.rs;
    q[row + x + L.GX] = v;
    for (unsigned m = xm; m; m &= m - 1) q[row + ghost_coord(__builtin_ctz(m), L.nx, L.Sx) + L.GX] = v;
  }
}


// ------------------------------------------------------------------ learned guess

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// SiLU(z) = z / (1 + 2^(-z log2 e)); exp2 overflows to inf for z below
// about -88, which gives the limit -0.
__device__ __forceinline__ float silu_f(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * -1.4426950408889634f));
}

// eight floats to bf16 (round to nearest even, four packed conversions)
__device__ __forceinline__ bf8 to_bf8(const f8& v) { return __builtin_convertvector(v, bf8); }

// The network evaluated for the 64 sites of a wave on the matrix cores
// (32x32x16 bf16 products, float32 accumulation).  Each layer computes
// H^T = W A^T, with units along M and sites along N (two tiles of 32 sites);
// lane l then holds units 8 (r/4) + 4 (l/32) + r%4 of site l%32 in
// accumulator register r.  Registers 0..7 and 8..15 of each output tile are
// used as they are as the B operands of two k-steps of the next layer (the
// weights are packed in the same unit order), so activations never leave
// their lanes.  Returns, in every lane, the standardised outputs of the
// lane's own site.  All 64 lanes must be active.
__device__ __forceinline__ void mlp_wave(const RlbmStepArgs& a, const float xin[9], float out[3]) {
  const int l = threadIdx.x & 63;
  const int half = l >> 5;
  // The weight pointers pass through an empty asm statement so that the
  // fragment loads stay at their use instead of being hoisted (which would
  // keep all fragments live).
  const unsigned short* fp = a.mlp_frag;
  const float* bp = a.mlp_bias;
  asm volatile("" : "+s"(fp), "+s"(bp));
  const bf8* __restrict__ fr = (const bf8*)fp;
  const v16f* __restrict__ br = (const v16f*)bp;
  auto frag = [&](int item) { return fr[item * 64 + l]; };
  auto bias = [&](int item) { return br[item * 64 + l]; };

  // layer-1 B operands (one k-step): inputs 8 half + e of site (l % 32) + 32 t
  bf8 bop[2][4];
  {
    // inputs 0..7 for half 0; input 8 and zeros for half 1 (selects, not
    // a lane-dependent register index)
    f8 own, oth;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float hi = e == 0 ? xin[8] : 0.0f;
      own[e] = half ? hi : xin[e];
      oth[e] = half ? xin[e] : hi;
    }
    f8 sw;
#pragma unroll
    for (int e = 0; e < 8; ++e) sw[e] = __shfl_xor(oth[e], 32);
    // tile t = half: own site; tile 1 - half: the partner lane's site
    const bf8 pown = to_bf8(own), psw = to_bf8(sw);
    bop[half ? 1 : 0][0] = pown;
    bop[half ? 0 : 1][0] = psw;
  }

  // hidden layers
  int ksteps = 1;
#pragma unroll
  for (int L = 0; L < 3; ++L) {
    bf8 nxt[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const v16f b0 = bias(RLBM_MLP_BFOFF[L] + m);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        v16f acc = b0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          if (s < ksteps)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(RLBM_MLP_FOFF[L] + m * RLBM_MLP_KSTEPS[L] + s),
                                                          bop[t][s], acc, 0, 0, 0);
        f8 lo, hi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          lo[e] = silu_f(acc[e]);
          hi[e] = silu_f(acc[8 + e]);
        }
        nxt[t][2 * m] = to_bf8(lo);
        nxt[t][2 * m + 1] = to_bf8(hi);
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) bop[t][s] = nxt[t][s];
    ksteps = 4;
  }

  // output layer: one tile of 32 rows (3 used)
  float res[2][3];
  const v16f b3 = bias(RLBM_MLP_BFOFF[3]);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    v16f acc = b3;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag(RLBM_MLP_FOFF[3] + s), bop[t][s], acc, 0, 0, 0);
    res[t][0] = acc[0];
    res[t][1] = acc[1];
    res[t][2] = acc[2];
  }
  // rows 0..2 live in lanes 0..31: tile 0 is theirs, tile 1 belongs to lane + 32
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    const float other = __shfl_xor(res[1][o], 32);
    out[o] = half ? other : res[0][o];
  }
}

// standardised inputs of a site from its float64 moments
__device__ __forceinline__ void mlp_inputs(const RlbmStepArgs& a, const double md[9], float xin[9]) {
  const double inv = 1.0 / md[0];
#pragma unroll
  for (int i = 0; i < 9; ++i) xin[i] = ((float)(md[i] * inv) - a.mlp_norm[i]) * a.mlp_norm[9 + i];
}

__device__ __forceinline__ void mlp_destandardise(const RlbmStepArgs& a, double n0, const float out[3], double& eps,
                                                  double& ux, double& uy) {
  eps = ((double)out[0] * a.mlp_norm[21] + a.mlp_norm[18]) * n0;
  ux = (double)out[1] * a.mlp_norm[22] + a.mlp_norm[19];
  uy = (double)out[2] * a.mlp_norm[23] + a.mlp_norm[20];
}

// ------------------------------------------------------------------ step

// Waves per SIMD requested from the register allocator: enough to overlap one
// wave's arithmetic with other waves' loads, while the class values of the
// largest stencils still fit in registers.
constexpr int step_waves(int qn, int p, bool g) {
  return g ? (p == RLBM_FP64 ? 1 : (qn <= 44 ? 3 : 2))
           : p == RLBM_FP64 ? (qn <= 48 ? 3 : 2) : (qn <= 48 ? 5 : 3);
}

// s_waitcnt operand that waits for LDS / scalar memory only (the vector
// memory and export counters at their maxima).
constexpr int kWaitLgkm0 = 0xC07F;

// Per-class table rows as whole structs, so each is fetched by wide scalar
// loads (moments: the nine monomials; equilibrium: M_j, n_j).
template <int P> struct Rows;
// (ml, el: the rows' rounding remainders, read by float32 storage only)
template <> struct Rows<RLBM_FP64> {
  struct alignas(16) M { double v[RLBM_ROWMD]; };
  struct alignas(16) E { double v[RLBM_ROWD]; };
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* m(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowmd;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* e(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->rowd;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* ml(TabPtr t) { return m(t); }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* el(TabPtr t) { return e(t); }
};
template <> struct Rows<RLBM_FP32_DEV> {
  struct alignas(16) M { float v[RLBM_ROWMF]; };
  struct alignas(16) E { float v[RLBM_ROWF]; };
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* m(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowmf;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* e(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->rowf;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* ml(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowmf_lo;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* el(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->rowf_lo;
  }
};
template <> struct Rows<RLBM_FP16_DEV> : Rows<RLBM_FP32_DEV> {};

template <typename R>
__device__ __forceinline__ R load_row(const __attribute__((address_space(4))) R* p) {
  R r;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(r.v) / sizeof(r.v[0])); ++i) r.v[i] = p->v[i];
  return r;
}

// Store of the post-collision value of class J for the fixed-stencil class
// code (float32 or float16 storage).
template <int P>
struct TileStore {
  __amdgpu_buffer_rsrc_t r;
  int vst;
  unsigned ob, ocs;  // own storage of class J at byte offset ob + J ocs
  template <int J>
  __device__ __forceinline__ void put(float v) {
    if constexpr (P == RLBM_FP32_DEV)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vst, ob + J * ocs, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, vst, ob + J * ocs,
                                            0);
  }
};

// Pulls of a generated stencil: offsets from the class displacements known at
// compile time and three per-lattice scalars, so no offset table is read.
template <class Fx, int P, class S, int... J>
__device__ __forceinline__ void pull_fixed(S (&raw)[sizeof...(J)], __amdgpu_buffer_rsrc_t r, int vld,
                                           const RlbmStepArgs& a, std::integer_sequence<int, J...>) {
  auto one = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const unsigned off = a.fo_base + j * a.fo_cs - Fx::kNy[j] * a.fo_rs - Fx::kNx[j] * a.fo_es;
    if constexpr (P == RLBM_FP32_DEV)
      raw[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vld, off, 0));
    else
      raw[j] = __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vld, off, 0));
  };
  (one(std::integral_constant<int, J>{}), ...);
}

// One time step for one tile per wave (kWave consecutive sites of a row), for
// a stencil of QMIN..QN classes.  The class loops are fully unrolled, so the
// populations stay in registers.
//
// Addressing: one buffer descriptor per tile and buffer, based at the lowest
// address any pull of the tile can reach, with 2^31 - 1 records; every class
// access adds a precomputed per-class scalar offset (from the offset table,
// below 2^31) to the shared lane offset.  Lanes past the row end re-read the
// row's last site, and their stores use the lane offset 2^31, beyond the
// records, which the hardware drops.  Classes Q <= j < QN (padding up to the
// kernel's class count; only j >= QMIN can be padding) read class 0's source,
// have all-zero table rows, and store through a descriptor with no records.
//
// Table rows: row j + 1 is requested right after the wait for row j, before
// class j is processed (scalar loads complete in any order, so every wait is
// for all of them).  In the FP16 mode the rows carry the per-class scale, so
// the kernel relaxes the stored ratios h_j = (f_j - f^ref_j) / f^ref_j directly.
template <int QN, int QMIN, int P, bool G, class Fx = void>
__global__ void __launch_bounds__(kStepBlock) __attribute__((amdgpu_waves_per_eu(step_waves(QN, P, G))))
k_step(RlbmStepArgs a) {
  constexpr bool kFixed = !std::is_same<Fx, void>::value;
  using SC = StepConsts<Fx>;
  using S = typename Traits<P>::S;
  using A = typename Traits<P>::A;
  typedef const __attribute__((address_space(4))) unsigned* OffPtr;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const int lane = (int)threadIdx.x & (kWave - 1);
  const int t = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (kStepBlock / kWave) +
                __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (t >= a.ntiles) return;  // whole wave
  const int Q = tb->c.Q;
  const int y = t / a.tiles_x;
  const int x0 = (t - y * a.tiles_x) * kWave;
  const int x = x0 + lane;
  const bool active = x < L.nx;
  const int nvalid = min(kWave, L.nx - x0);
  const long long lo = (long long)(y + L.GY - L.Sy) * L.rs + L.GX - L.Sx + x0;
  const __amdgpu_buffer_rsrc_t rs_ld = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((const char*)a.src + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rs_st = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((char*)a.dst + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rs_none = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((char*)a.dst + lo * (long long)sizeof(S)), (short)0, 0, kRsrcWord3);
  const int vld = min(lane, nvalid - 1) * (int)sizeof(S);
  const int vst = active ? lane * (int)sizeof(S) : kRecOut;
  const OffPtr pull = (OffPtr)a.offs;
  const OffPtr own = (OffPtr)a.offs_st;

  // pull: f_j(x, t) = f*_j(x - n_j, t - 1) (exact streaming)
  S raw[QN];
  if constexpr (kFixed) {
    pull_fixed<Fx, P>(raw, rs_ld, vld, a, std::make_integer_sequence<int, QN>{});
  } else {
#pragma unroll
  for (int j = 0; j < QN; ++j) {
    if constexpr (P == RLBM_FP64)
      raw[j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs_ld, vld, pull[j], 0));
    else if constexpr (P == RLBM_FP32_DEV)
      raw[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_ld, vld, pull[j], 0));
    else
      raw[j] = __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs_ld, vld, pull[j], 0));
  }
  }

  // moments (eq. mj-discrete-second-moment) as one multiply-add per
  // monomial; deviation modes add the exact float64 moments of the reference
  // float32 storage: m collects the float parts of the rows, ml their
  // rounding remainders (the rows to about 2^-48; zero in the other modes)
  constexpr bool kSplit = P == RLBM_FP32_DEV;
  A f[QN];
  A m[9] = {A(0), A(0), A(0), A(0), A(0), A(0), A(0), A(0), A(0)};
  A ml[9] = {A(0), A(0), A(0), A(0), A(0), A(0), A(0), A(0), A(0)};
  if constexpr (kFixed) {
#pragma unroll
    for (int j = 0; j < QN; ++j) f[j] = (A)raw[j];
    Fx::moments(f, m, ml);
  } else {
    const auto* rows = Rows<P>::m(tb);
    const auto* rows_lo = Rows<P>::ml(tb);
    typename Rows<P>::M cur = load_row(rows);
    typename Rows<P>::M cur_lo = kSplit ? load_row(rows_lo) : cur;
#pragma unroll
    for (int j = 0; j < QN; ++j) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      const int jn = j + 1 < QN ? j + 1 : j;
      const typename Rows<P>::M nxt = load_row(rows + jn);
      const typename Rows<P>::M nxt_lo = kSplit ? load_row(rows_lo + jn) : nxt;
      __builtin_amdgcn_sched_barrier(0);
      f[j] = (A)raw[j];
#pragma unroll
      for (int k = 0; k < 9; ++k) m[k] = fma(f[j], (A)cur.v[k], m[k]);
      if constexpr (kSplit) {
#pragma unroll
        for (int k = 0; k < 9; ++k) ml[k] = fma(f[j], (A)cur_lo.v[k], ml[k]);
      }
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
      cur_lo = nxt_lo;
    }
  }
  // all nine sums are formed here, next to the class values (not sunk past
  // the Landau solve, which would re-fetch the rows)
#pragma unroll
  for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(m[k]));
  if constexpr (kSplit) {
#pragma unroll
    for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(ml[k]));
  }
  // past its pulls, a wave issues ahead of waves still waiting for theirs, so
  // it finishes and frees its slot sooner
  __builtin_amdgcn_s_setprio(2);
  double md[9];
#pragma unroll
  for (int k = 0; k < 9; ++k)
    md[k] = (P == RLBM_FP64) ? (double)m[k] : SC::ref_mom(tb, k) + ((double)m[k] + (double)ml[k]);

  double e0 = 0.0, ux0 = 0.0, uy0 = 0.0;
  const long long wsite = (long long)y * L.nx + min(x, L.nx - 1);
  if constexpr (G) {
    float xin[9], yo[3];
    mlp_inputs(a, md, xin);
    mlp_wave(a, xin, yo);
    mlp_destandardise(a, md[0], yo, e0, ux0, uy0);
  } else if (a.warm) {  // the frame this site converged to in the previous step
    e0 = a.warm[wsite];
    ux0 = a.warm[wsite + a.warm_plane];
    uy0 = a.warm[wsite + 2 * a.warm_plane];
  }
  Macro mac = macroscopic_z(tb, SC::zeta(tb), SC::inv_zeta(tb), md[0], md[1], md[2], md[3], md[4], md[5], md[6],
                            md[7], md[8], a.landau_tol, a.landau_maxit, a.landau_method, e0, ux0, uy0);
  if constexpr (!G) {
    if (a.warm && active) {
      a.warm[wsite] = (float)mac.eps;
      a.warm[wsite + a.warm_plane] = (float)mac.ux;
      a.warm[wsite + 2 * a.warm_plane] = (float)mac.uy;
    }
  }
  const double tau = a.tau_mode == RLBM_TAU_CONST ? a.tau : tau_eta_over_s(a.tk1, a.tk2, mac.n, mac.T);
  double b[RLBM_NB];
  projections(SC::proj(tb), mac.T, mac.R, mac.gamma, mac.gamma * mac.ux, mac.gamma * mac.uy, b);
  // Anderson-Witting frequency p_i.U/(p_i^0 tau) = gamma (1 - v0 n_i.u)/tau (eq. discrete-relativistic-boltzmann)
  const double w0 = a.tau_mode == RLBM_TAU_CONST ? mac.gamma * a.inv_tau : div_nr(mac.gamma, tau);
  const double wx = -w0 * SC::v0(tb) * mac.ux, wy = -w0 * SC::v0(tb) * mac.uy;
  A nb[RLBM_NB];
#pragma unroll
  for (int k = 0; k < RLBM_NB; ++k) nb[k] = (A)(mac.n * b[k] - (P == RLBM_FP64 ? 0.0 : SC::nb_ref(tb, k)));
  const A W0 = (A)w0, WX = (A)wx, WY = (A)wy;

  // equilibrium (eq. mj-discrete-feq) and relaxation, stored at the own site
  if constexpr (kFixed) {
    TileStore<P> st{rs_st, vst, a.fo_base, a.fo_cs};
    Fx::collide(f, nb, W0, WX, WY, st);
  } else {
    const auto* rows = Rows<P>::e(tb);
    const auto* rows_lo = Rows<P>::el(tb);
    typename Rows<P>::E cur = load_row(rows);
    typename Rows<P>::E cur_lo = kSplit ? load_row(rows_lo) : cur;
#pragma unroll
    for (int j = 0; j < QN; ++j) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      const int jn = j + 1 < QN ? j + 1 : j;
      const typename Rows<P>::E nxt = load_row(rows + jn);
      const typename Rows<P>::E nxt_lo = kSplit ? load_row(rows_lo + jn) : nxt;
      __builtin_amdgcn_sched_barrier(0);
      A feq = nb[0] * (A)cur.v[0];
#pragma unroll
      for (int k = 1; k < RLBM_NB; ++k) feq = fma(nb[k], (A)cur.v[k], feq);
      const A om = fma(WY, (A)cur.v[RLBM_R_NY], fma(WX, (A)cur.v[RLBM_R_NX], W0));
      A diff = f[j] - feq;
      if constexpr (kSplit) {
        // the remainder part of f^eq, taken off the small difference f - f^eq
        A feql = nb[0] * (A)cur_lo.v[0];
#pragma unroll
        for (int k = 1; k < RLBM_NB; ++k) feql = fma(nb[k], (A)cur_lo.v[k], feql);
        diff = diff - feql;
      }
      f[j] = fma(-om, diff, f[j]);
      const __amdgpu_buffer_rsrc_t r = (j < QMIN || j < Q) ? rs_st : rs_none;
      if constexpr (P == RLBM_FP64)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, f[j]), r, vst, own[j], 0);
      else if constexpr (P == RLBM_FP32_DEV)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, f[j]), r, vst, own[j], 0);
      else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)f[j]), r, vst, own[j], 0);
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
      cur_lo = nxt_lo;
    }
  }

  // ghost copies are needed only near the lattice edges (uniform test)
  const unsigned ym = (y < L.Sy || y >= L.ny - L.Sy) ? ghost_mask(y, L.ny, L.Sy, L.bc_y) : 0u;
  const bool xedge = x0 < L.Sx || x0 + kWave > L.nx - L.Sx;
  if (xedge || ym != 0u) {
    S* __restrict__ dst = (S*)a.dst;
    const unsigned xm = xedge ? ghost_mask(x, L.nx, L.Sx, L.bc_x) : 0u;
    if (active) {
#pragma unroll
      for (int j = 0; j < QN; ++j)
        if (j < Q) store_ghosts(dst + (long long)j * L.cs, L, x, y, xm, ym, (S)f[j]);
    }
  }
  wave_stats(a.slots, t, active ? mac.flags : 0u, active ? (unsigned)mac.iters : 0u,
             active ? (unsigned)mac.iters : 0u);
}

// ------------------------------------------------------------------ 3D step
//
// 3D lattices (Sec. V: the method runs in three dimensions as in two): every
// population of the stencil is its own class, moments are the 14 components
// of N^a and T^ab, the Landau frame has three velocity components (Newton on
// the quartic characteristic polynomial), the equilibrium takes all 14
// projections, and streaming moves a population by its 3D vector.  Layout:
// storage planes z of storage rows y, each row holding the Q class rows of
// one lattice row (x fastest), with ghost columns, rows and planes of the
// stencil's reach on every side.  One wave per 64 sites of a row, one buffer
// descriptor per tile based at the lowest element its pulls reach, per-class
// byte offsets from the context's table (class offsets in 3D include n_z).

// ghost copies of site (x, y, z) in class row q: every combination of the
// owner or ghost coordinate on each axis except the owner itself
template <typename S>
__device__ __forceinline__ void store_ghosts3(S* __restrict__ q, const RlbmLayout& L, int x, int y, int z,
                                              unsigned xm, unsigned ym, unsigned zm, S v) {
  // bit 0: the owner coordinate, bit i + 1: ghost coordinate i (up to 2 x 16
  // ghosts per axis, so 33 bits)
  typedef unsigned long long M64;
  const M64 zall = ((M64)zm << 1) | 1ull, yall = ((M64)ym << 1) | 1ull, xall = ((M64)xm << 1) | 1ull;
  for (M64 mz = zall; mz; mz &= mz - 1) {
    const int bz = __builtin_ctzll(mz);
    const int cz = bz == 0 ? z : ghost_coord(bz - 1, L.nz, L.Sz);
    for (M64 my = yall; my; my &= my - 1) {
      const int by = __builtin_ctzll(my);
      const int cy = by == 0 ? y : ghost_coord(by - 1, L.ny, L.Sy);
      const long long row = (long long)(cz + L.GZ) * L.zs + (long long)(cy + L.GY) * L.rs + L.GX;
      for (M64 mx = xall; mx; mx &= mx - 1) {
        const int bx = __builtin_ctzll(mx);
        if (bx == 0 && by == 0 && bz == 0) continue;
        const int cx = bx == 0 ? x : ghost_coord(bx - 1, L.nx, L.Sx);
        q[row + cx] = v;
      }
    }
  }
}

template <int P> struct Rows3;
static_assert(RLBM_ROW3 * sizeof(float) % 16 == 0 && RLBM_ROWM3 * sizeof(float) % 16 == 0,
              "3D table rows must be whole 16-byte structs");
static_assert(RLBM_ROWF * sizeof(float) % 16 == 0 && RLBM_ROWMF * sizeof(float) % 16 == 0 &&
                  RLBM_ROWD * sizeof(double) % 16 == 0 && RLBM_ROWMD * sizeof(double) % 16 == 0,
              "2D table rows must be whole 16-byte structs");
template <> struct Rows3<RLBM_FP64> {
  struct alignas(16) M { double v[RLBM_ROWM3]; };
  struct alignas(16) E { double v[RLBM_ROW3]; };
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* m(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowm3d;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* e(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->row3d;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* ml(TabPtr t) { return m(t); }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* el(TabPtr t) { return e(t); }
};
template <> struct Rows3<RLBM_FP32_DEV> {
  struct alignas(16) M { float v[RLBM_ROWM3]; };
  struct alignas(16) E { float v[RLBM_ROW3]; };
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* m(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowm3f;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* e(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->row3f;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) M* ml(TabPtr t) {
    return (const __attribute__((address_space(4))) M*)t->rowm3f_lo;
  }
  static __device__ __forceinline__ const __attribute__((address_space(4))) E* el(TabPtr t) {
    return (const __attribute__((address_space(4))) E*)t->row3f_lo;
  }
};
template <> struct Rows3<RLBM_FP16_DEV> : Rows3<RLBM_FP32_DEV> {};

constexpr int step3_waves(int qn, int p) { return p == RLBM_FP64 ? (qn <= 60 ? 2 : 1) : (qn <= 60 ? 3 : 2); }

// Store of the post-collision value of population J for the generated 3D
// code (float32 or float16 storage), at the offset-table entry of J.
template <int P>
struct TileStore3 {
  __amdgpu_buffer_rsrc_t r;
  int vst;
  const __attribute__((address_space(4))) unsigned* own;
  template <int J>
  __device__ __forceinline__ void put(float v) {
    if constexpr (P == RLBM_FP32_DEV)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vst, own[J], 0);
    else
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, vst, own[J], 0);
  }
};

// Fx: generated sign-orbit code of a configured 3D stencil (float32 or
// float16 storage; rlbm_fixed_stencils.h), or void for the table-driven
// class loops.
template <int QN, int QMIN, int P, class Fx = void>
__global__ void __launch_bounds__(kStepBlock) __attribute__((amdgpu_waves_per_eu(step3_waves(QN, P))))
k_step3(RlbmStepArgs a) {
  constexpr bool kFixed = !std::is_same<Fx, void>::value;
  using S = typename Traits<P>::S;
  using A = typename Traits<P>::A;
  typedef const __attribute__((address_space(4))) unsigned* OffPtr;
  constexpr bool kSplit = P == RLBM_FP32_DEV;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const int lane = (int)threadIdx.x & (kWave - 1);
  const int t = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (kStepBlock / kWave) +
                __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (t >= a.ntiles) return;  // whole wave
  const int Q = tb->c.Q;
  const int row = t / a.tiles_x;  // z * ny + y
  const int z = row / L.ny, y = row - z * L.ny;
  const int x0 = (t - row * a.tiles_x) * kWave;
  const int x = x0 + lane;
  const bool active = x < L.nx;
  const int nvalid = min(kWave, L.nx - x0);
  const long long lo =
      (long long)(z + L.GZ - L.Sz) * L.zs + (long long)(y + L.GY - L.Sy) * L.rs + L.GX - L.Sx + x0;
  const __amdgpu_buffer_rsrc_t rs_ld = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((const char*)a.src + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rs_st = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((char*)a.dst + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rs_none = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((char*)a.dst + lo * (long long)sizeof(S)), (short)0, 0, kRsrcWord3);
  const int vld = min(lane, nvalid - 1) * (int)sizeof(S);
  const int vst = active ? lane * (int)sizeof(S) : kRecOut;
  const OffPtr pull = (OffPtr)a.offs;
  const OffPtr own = (OffPtr)a.offs_st;

  // pull: f_i(x, t) = f*_i(x - n_i, t - 1) (exact streaming)
  S raw[QN];
#pragma unroll
  for (int j = 0; j < QN; ++j) {
    if constexpr (P == RLBM_FP64)
      raw[j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs_ld, vld, pull[j], 0));
    else if constexpr (P == RLBM_FP32_DEV)
      raw[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_ld, vld, pull[j], 0));
    else
      raw[j] = __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs_ld, vld, pull[j], 0));
  }

  // the 14 moments (float32 storage: rows plus rounding remainders)
  A f[QN];
  A m[RLBM_NB3], ml[RLBM_NB3];
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k) m[k] = ml[k] = A(0);
  if constexpr (kFixed) {
#pragma unroll
    for (int j = 0; j < QN; ++j) f[j] = (A)raw[j];
    Fx::moments(f, m, ml);
  } else {
    const auto* rows = Rows3<P>::m(tb);
    const auto* rows_lo = Rows3<P>::ml(tb);
    typename Rows3<P>::M cur = load_row(rows);
    typename Rows3<P>::M cur_lo = kSplit ? load_row(rows_lo) : cur;
#pragma unroll
    for (int j = 0; j < QN; ++j) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      const int jn = j + 1 < QN ? j + 1 : j;
      const typename Rows3<P>::M nxt = load_row(rows + jn);
      const typename Rows3<P>::M nxt_lo = kSplit ? load_row(rows_lo + jn) : nxt;
      __builtin_amdgcn_sched_barrier(0);
      f[j] = (A)raw[j];
#pragma unroll
      for (int k = 0; k < RLBM_NB3; ++k) m[k] = fma(f[j], (A)cur.v[k], m[k]);
      if constexpr (kSplit) {
#pragma unroll
        for (int k = 0; k < RLBM_NB3; ++k) ml[k] = fma(f[j], (A)cur_lo.v[k], ml[k]);
      }
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
      cur_lo = nxt_lo;
    }
  }
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k) asm volatile("" : "+v"(m[k]));
  if constexpr (kSplit) {
#pragma unroll
    for (int k = 0; k < RLBM_NB3; ++k) asm volatile("" : "+v"(ml[k]));
  }
  __builtin_amdgcn_s_setprio(2);
  double md[RLBM_NB3];
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k)
    md[k] = (P == RLBM_FP64) ? (double)m[k] : tb->c.ref_mom3[k] + ((double)m[k] + (double)ml[k]);

  // Landau frame, density, EOS
  unsigned flags = 0;
  double eps, u[3];
  const int iters = landau_newton3(md, newton_thresh(a.landau_tol), a.landau_maxit, eps, u, md[4]);
  if (iters > a.landau_maxit) flags |= RLBM_H_LANDAU;
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (!(u2 < 1.0)) flags |= RLBM_H_SUPERLUMINAL;
  const double gamma = rsqrt_nr(1.0 - u2);
  const double n = gamma * (md[0] - u[0] * md[1] - u[1] * md[2] - u[2] * md[3]);
  if (!(n > 0.0) || !(eps > 0.0)) flags |= RLBM_H_RANGE;
  const double e = div_nr(eps, n);
  const double T = eos_temperature_tab(tb, e, tb->c.zeta, flags);
  const double R = (e - 3.0 * T) * tb->c.inv_zeta;
  if (!isfinite(T) || !isfinite(eps) || !isfinite(n) || !isfinite(R)) flags |= RLBM_H_NAN;
  const double tau = a.tau_mode == RLBM_TAU_CONST ? a.tau : tau_eta_over_s(a.tk1, a.tk2, n, T);
  double b[RLBM_NB3];
  const double U[3] = {gamma * u[0], gamma * u[1], gamma * u[2]};
  projections3(proj_consts(tb), T, R, gamma, U, b);
  const double w0 = a.tau_mode == RLBM_TAU_CONST ? gamma * a.inv_tau : div_nr(gamma, tau);
  const double v0 = tb->c.v0;
  A nb[RLBM_NB3];
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k) nb[k] = (A)(n * b[k] - (P == RLBM_FP64 ? 0.0 : tb->c.nb_ref3[k]));
  const A W0 = (A)w0, WX = (A)(-w0 * v0 * u[0]), WY = (A)(-w0 * v0 * u[1]), WZ = (A)(-w0 * v0 * u[2]);

  // equilibrium (eq. mj-discrete-feq, all 14 polynomials) and relaxation
  if constexpr (kFixed) {
    TileStore3<P> st{rs_st, vst, own};
    Fx::collide(f, nb, W0, WX, WY, WZ, st);
  } else {
    const auto* rows = Rows3<P>::e(tb);
    const auto* rows_lo = Rows3<P>::el(tb);
    typename Rows3<P>::E cur = load_row(rows);
    typename Rows3<P>::E cur_lo = kSplit ? load_row(rows_lo) : cur;
#pragma unroll
    for (int j = 0; j < QN; ++j) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
      const int jn = j + 1 < QN ? j + 1 : j;
      const typename Rows3<P>::E nxt = load_row(rows + jn);
      const typename Rows3<P>::E nxt_lo = kSplit ? load_row(rows_lo + jn) : nxt;
      __builtin_amdgcn_sched_barrier(0);
      A feq = nb[0] * (A)cur.v[0];
#pragma unroll
      for (int k = 1; k < RLBM_NB3; ++k) feq = fma(nb[k], (A)cur.v[k], feq);
      const A om = fma(WZ, (A)cur.v[RLBM_R3_NZ], fma(WY, (A)cur.v[RLBM_R3_NY], fma(WX, (A)cur.v[RLBM_R3_NX], W0)));
      A diff = f[j] - feq;
      if constexpr (kSplit) {
        A feql = nb[0] * (A)cur_lo.v[0];
#pragma unroll
        for (int k = 1; k < RLBM_NB3; ++k) feql = fma(nb[k], (A)cur_lo.v[k], feql);
        diff = diff - feql;
      }
      f[j] = fma(-om, diff, f[j]);
      const __amdgpu_buffer_rsrc_t r = (j < QMIN || j < Q) ? rs_st : rs_none;
      if constexpr (P == RLBM_FP64)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, f[j]), r, vst, own[j], 0);
      else if constexpr (P == RLBM_FP32_DEV)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, f[j]), r, vst, own[j], 0);
      else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)f[j]), r, vst, own[j], 0);
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
      cur_lo = nxt_lo;
    }
  }

  // ghost copies near the lattice edges
  const unsigned zm = (z < L.Sz || z >= L.nz - L.Sz) ? ghost_mask(z, L.nz, L.Sz, L.bc_z) : 0u;
  const unsigned ym = (y < L.Sy || y >= L.ny - L.Sy) ? ghost_mask(y, L.ny, L.Sy, L.bc_y) : 0u;
  const bool xedge = x0 < L.Sx || x0 + kWave > L.nx - L.Sx;
  if (xedge || ym != 0u || zm != 0u) {
    S* __restrict__ dst = (S*)a.dst;
    const unsigned xm = xedge ? ghost_mask(x, L.nx, L.Sx, L.bc_x) : 0u;
    if (active) {
#pragma unroll
      for (int j = 0; j < QN; ++j)
        if (j < Q) store_ghosts3(dst + (long long)j * L.cs, L, x, y, z, xm, ym, zm, (S)f[j]);
    }
  }
  wave_stats(a.slots, t, active ? flags : 0u, active ? (unsigned)iters : 0u, active ? (unsigned)iters : 0u);
}

// Third-order step (float64 storage; every dimension runs on the 3D
// layout, merged classes included).  Two passes over the populations: the
// first pulls them (exact streaming) and sums the 14 moments; the second
// pulls them again (the same addresses, now in cache), forms each
// equilibrium from the 30 projections on the centred, scaled monomials and
// the population's row (eq. mj-projected-distribution at N = 3), relaxes and
// stores.  No
// population stays in registers, so any class count fits.
constexpr int kO3Chunk = 8;

// D: the stencil's class dimension (1, 2: merged classes, only the moments
// and equilibrium terms that can be nonzero; 3: every population).
// P: float64 storage, or float32 deviations d = f - f^ref (sums in float32
// over hi + lo rows, the reference's moments and projections added in
// float64, as in the second-order float32 step).
// Pulls and stores of the generated third-order code (by class index, at
// the offset-table entries; stores also write the ghost copies near the
// lattice edges).
template <int P>
struct PullO3 {
  using A = typename Traits<P>::A;
  __amdgpu_buffer_rsrc_t r;
  int vld;
  const __attribute__((address_space(4))) unsigned* pull;
  template <int J>
  __device__ __forceinline__ A get() const {
    if constexpr (P == RLBM_FP32_DEV)
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vld, pull[J], 0));
    else
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vld, pull[J], 0));
  }
};
template <int P>
struct StoreO3 {
  using A = typename Traits<P>::A;
  using S = typename Traits<P>::S;
  __amdgpu_buffer_rsrc_t r;
  int vst;
  const __attribute__((address_space(4))) unsigned* own;
  bool ghosts;  // the tile touches a lattice edge and the lane holds a site
  S* dst;
  RlbmLayout L;
  int x, y, z;
  unsigned xm, ym, zm;
  template <int J>
  __device__ __forceinline__ void put(A v) {
    if constexpr (P == RLBM_FP32_DEV)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vst, own[J], 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), r, vst, own[J], 0);
    if (ghosts) store_ghosts3(dst + (long long)J * L.cs, L, x, y, z, xm, ym, zm, (S)v);
  }
};

// Fx: generated orbit code of the configured third-order stencil
// (rlbm_fixed_stencils.h), or void for the table-driven passes.  The
// generated code is held to four waves per SIMD in float32 (it would
// otherwise take up to 157 registers per lane for the orbits' straight-line
// code) and to two in 3D float64 (one otherwise); measured, the 2D float64
// code runs best with its own choice (two waves).
template <int D, int P, class Fx = void>
__global__ void __launch_bounds__(kStepBlock)
    __attribute__((amdgpu_waves_per_eu(std::is_same<Fx, void>::value ? 1 : (P == RLBM_FP32_DEV ? 4 : (D == 3 ? 2 : 1)))))
    k_step_o3(RlbmStepArgs a) {
  typedef const __attribute__((address_space(4))) unsigned* OffPtr;
  using S = typename Traits<P>::S;
  using A = typename Traits<P>::A;
  constexpr bool kFixed = !std::is_same<Fx, void>::value;
  constexpr bool kF32 = P == RLBM_FP32_DEV;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const int lane = (int)threadIdx.x & (kWave - 1);
  const int t = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (kStepBlock / kWave) +
                __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (t >= a.ntiles) return;  // whole wave
  const int Q = tb->c.Q;
  const int row = t / a.tiles_x;  // z * ny + y
  const int z = row / L.ny, y = row - z * L.ny;
  const int x0 = (t - row * a.tiles_x) * kWave;
  const int x = x0 + lane;
  const bool active = x < L.nx;
  const int nvalid = min(kWave, L.nx - x0);
  const long long lo =
      (long long)(z + L.GZ - L.Sz) * L.zs + (long long)(y + L.GY - L.Sy) * L.rs + L.GX - L.Sx + x0;
  const __amdgpu_buffer_rsrc_t rs_ld = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((const char*)a.src + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rs_st = __builtin_amdgcn_make_buffer_rsrc(
      (void*)((char*)a.dst + lo * (long long)sizeof(S)), (short)0, kRecAll, kRsrcWord3);
  const int vld = min(lane, nvalid - 1) * (int)sizeof(S);
  const int vst = active ? lane * (int)sizeof(S) : kRecOut;
  const OffPtr pull = (OffPtr)a.offs;
  const OffPtr own = (OffPtr)a.offs_st;
  auto pull_one = [&](int j) -> A {
    if constexpr (kF32)
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_ld, vld, pull[j], 0));
    else
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs_ld, vld, pull[j], 0));
  };

  // populations go in chunks of kO3Chunk: all pulls of a chunk are issued
  // before the first is used (a class-by-class loop would wait out one
  // memory round trip per class); the last chunk re-reads class Q - 1
  A m[RLBM_NB3], ml[RLBM_NB3];
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k) m[k] = ml[k] = A(0);
  if constexpr (kFixed) {
    PullO3<P> pl{rs_ld, vld, pull};
    Fx::moments(pl, m, ml);
  } else {
  for (int j0 = 0; j0 < Q; j0 += kO3Chunk) {
    A f[kO3Chunk];
#pragma unroll
    for (int i = 0; i < kO3Chunk; ++i) f[i] = pull_one(min(j0 + i, Q - 1));
#pragma unroll
    for (int i = 0; i < kO3Chunk; ++i) {
      const int j = min(j0 + i, Q - 1);
      const A fi = j0 + i < Q ? f[i] : A(0);
#pragma unroll
      for (int k = 0; k < RLBM_NB3; ++k) {
        if (!o3_mom_active(D, k)) continue;
        if constexpr (kF32) {
          m[k] = fmaf(fi, tb->rowm3f[j][k], m[k]);
          ml[k] = fmaf(fi, tb->rowm3f_lo[j][k], ml[k]);
        } else {
          m[k] = fma(fi, tb->rowm3d[j][k], m[k]);
        }
      }
      // (keeps the scalar row loads of later classes from piling up in SGPRs)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  }
  double md[RLBM_NB3];
#pragma unroll
  for (int k = 0; k < RLBM_NB3; ++k)
    md[k] = kF32 ? tb->c.ref_mom3[k] + ((double)m[k] + (double)ml[k]) : (double)m[k];

  // Landau frame, density, EOS
  unsigned flags = 0;
  double eps, u[3];
  const int iters = landau_newton3(md, newton_thresh(a.landau_tol), a.landau_maxit, eps, u, md[4]);
  if (iters > a.landau_maxit) flags |= RLBM_H_LANDAU;
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (!(u2 < 1.0)) flags |= RLBM_H_SUPERLUMINAL;
  const double gamma = rsqrt_nr(1.0 - u2);
  const double n = gamma * (md[0] - u[0] * md[1] - u[1] * md[2] - u[2] * md[3]);
  if (!(n > 0.0) || !(eps > 0.0)) flags |= RLBM_H_RANGE;
  const double T = eos_temperature_tab(tb, div_nr(eps, n), tb->c.zeta, flags);
  if (!isfinite(T) || !isfinite(eps) || !isfinite(n)) flags |= RLBM_H_NAN;
  const double tau = a.tau_mode == RLBM_TAU_CONST ? a.tau : tau_eta_over_s(a.tk1, a.tk2, n, T);
  const double U[4] = {gamma, gamma * u[0], gamma * u[1], gamma * u[2]};
  double Mr[RLBM_NO3], Md[RLBM_NO3];
  mj_moments_o3(n, eps, n * T, T, tb->c.inv_zeta, tb->c.zeta, U, Mr);
  centred_o3(Mr, tb->c.o3_c, tb->c.o3_is0, tb->c.o3_isp, Md);
  A M[RLBM_NO3];
#pragma unroll
  for (int k = 0; k < RLBM_NO3; ++k) M[k] = (A)(kF32 ? Md[k] - tb->c.o3_aref[k] : Md[k]);
  const double w0 = a.tau_mode == RLBM_TAU_CONST ? gamma * a.inv_tau : div_nr(gamma, tau);
  const double v0 = tb->c.v0;
  const A W0 = (A)w0, WX = (A)(-w0 * v0 * u[0]), WY = (A)(-w0 * v0 * u[1]), WZ = (A)(-w0 * v0 * u[2]);

  const unsigned zm = (z < L.Sz || z >= L.nz - L.Sz) ? ghost_mask(z, L.nz, L.Sz, L.bc_z) : 0u;
  const unsigned ym = (y < L.Sy || y >= L.ny - L.Sy) ? ghost_mask(y, L.ny, L.Sy, L.bc_y) : 0u;
  const bool xedge = x0 < L.Sx || x0 + kWave > L.nx - L.Sx;
  const bool ghosts = xedge || ym != 0u || zm != 0u;
  const unsigned xm = xedge ? ghost_mask(x, L.nx, L.Sx, L.bc_x) : 0u;
  S* __restrict__ dst = (S*)a.dst;
  if constexpr (kFixed) {
    // an opaque copy of the lane offset, so that the second pulls are not
    // merged with the first ones (which would keep every population in
    // registers across the Landau solve)
    int vld2 = vld;
    asm volatile("" : "+v"(vld2));
    PullO3<P> pl{rs_ld, vld2, pull};
    StoreO3<P> st{rs_st, vst, own, ghosts && active, dst, L, x, y, z, xm, ym, zm};
    Fx::collide(pl, M, W0, WX, WY, WZ, st);
  } else {
  for (int j0 = 0; j0 < Q; j0 += kO3Chunk) {
    A f[kO3Chunk];
#pragma unroll
    for (int i = 0; i < kO3Chunk; ++i) f[i] = pull_one(min(j0 + i, Q - 1));
#pragma unroll
    for (int i = 0; i < kO3Chunk; ++i) {
      const int j = j0 + i;
      if (j >= Q) break;
      constexpr O3Act act = kO3Act[D];
      A diff, om;
      if constexpr (kF32) {
        const auto& r = tb->rowo3f[j];
        const auto& rl = tb->rowo3f_lo[j];
        float feq = M[act.m[0]] * r[0], feql = M[act.m[0]] * rl[0];
#pragma unroll
        for (int k = 1; k < act.n; ++k) {
          feq = fmaf(M[act.m[k]], r[k], feq);
          feql = fmaf(M[act.m[k]], rl[k], feql);
        }
        diff = (f[i] - feq) - feql;
        om = fmaf(WX, r[RLBM_RO3_NX], W0);
        if (D >= 2) om = fmaf(WY, r[RLBM_RO3_NY], om);
        if (D == 3) om = fmaf(WZ, r[RLBM_RO3_NZ], om);
      } else {
        const auto& r = tb->rowo3[j];
        double feq = M[act.m[0]] * r[0];
#pragma unroll
        for (int k = 1; k < act.n; ++k) feq = fma(M[act.m[k]], r[k], feq);
        diff = f[i] - feq;
        om = fma(WX, r[RLBM_RO3_NX], W0);
        if (D >= 2) om = fma(WY, r[RLBM_RO3_NY], om);
        if (D == 3) om = fma(WZ, r[RLBM_RO3_NZ], om);
      }
      const A out = fma(-om, diff, f[i]);
      if constexpr (kF32)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, out), rs_st, vst, own[j], 0);
      else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, out), rs_st, vst, own[j], 0);
      if (ghosts && active) store_ghosts3(dst + (long long)j * L.cs, L, x, y, z, xm, ym, zm, (S)out);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  }
  wave_stats(a.slots, t, active ? flags : 0u, active ? (unsigned)iters : 0u, active ? (unsigned)iters : 0u);
}

// f_i(x, 0) = f_i^eq(n, T, u) at third order (D, P as in k_step_o3; float32
// storage keeps f^eq - f^ref = R . (a - a^ref))
template <int D, int P>
__global__ void __launch_bounds__(kBlock) k_init_o3(RlbmInitArgs a, const double* __restrict__ uz) {
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long site = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (site >= (long long)L.nx * L.ny * L.nz) return;
  const int x = (int)(site % L.nx);
  const long long yz = site / L.nx;
  const int y = (int)(yz % L.ny), z = (int)(yz / L.ny);
  const double n = a.n[site], T = a.T[site];
  const double u[3] = {a.ux[site], a.uy[site], uz ? uz[site] : 0.0};
  const double g = 1.0 / sqrt(1.0 - u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
  const double U[4] = {g, g * u[0], g * u[1], g * u[2]};
  const double eps = n * (3.0 * T + tb->c.zeta * k1k2_ratio(tb->c.zeta / T));
  double Mr[RLBM_NO3], M[RLBM_NO3];
  mj_moments_o3(n, eps, n * T, T, tb->c.inv_zeta, tb->c.zeta, U, Mr);
  centred_o3(Mr, tb->c.o3_c, tb->c.o3_is0, tb->c.o3_isp, M);
  const long long o = (long long)(z + L.GZ) * L.zs + (long long)(y + L.GY) * L.rs + x + L.GX;
  constexpr O3Act act = kO3Act[D];
  if (P == RLBM_FP32_DEV)
    for (int k = 0; k < RLBM_NO3; ++k) M[k] -= tb->c.o3_aref[k];
  for (int j = 0; j < tb->c.Q; ++j) {
    double fe = 0.0;
#pragma unroll
    for (int k = 0; k < act.n; ++k) fe = fma(M[act.m[k]], tb->rowo3[j][k], fe);
    if (P == RLBM_FP32_DEV)
      ((float*)a.dst)[(long long)j * L.cs + o] = (float)fe;
    else
      ((double*)a.dst)[(long long)j * L.cs + o] = fe;
  }
}

// 3D fields and raw moments of the current (pre-collision) state
template <int P>
__global__ void __launch_bounds__(kBlock) k_moments3(RlbmMomArgs a, double* __restrict__ uz,
                                                     double* __restrict__ raw14) {
  using S = typename Traits<P>::S;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long S3 = (long long)L.nx * L.ny * L.nz;
  const long long site = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (site >= S3) return;
  const int x = (int)(site % L.nx);
  const long long yz = site / L.nx;
  const int y = (int)(yz % L.ny), z = (int)(yz / L.ny);
  const S* __restrict__ src = (const S*)a.src;
  double m[RLBM_NB3] = {};
  for (int j = 0; j < tb->c.Q; ++j) {
    const int sx = a.shift ? x - tb->nx[j] : x, sy = a.shift ? y - tb->ny[j] : y, sz = a.shift ? z - tb->nz[j] : z;
    const long long idx = (long long)j * L.cs + (long long)(sz + L.GZ) * L.zs + (long long)(sy + L.GY) * L.rs + sx + L.GX;
    const double f = (double)to_arith<P>(src[idx], tb, j);
    for (int k = 0; k < RLBM_NB3; ++k) m[k] = fma(f, tb->rowm3d[j][k], m[k]);
  }
  if (P != RLBM_FP64)
    for (int k = 0; k < RLBM_NB3; ++k) m[k] += tb->c.ref_mom3[k];
  unsigned flags = 0;
  double eps, u[3];
  (void)landau_newton3(m, newton_thresh(a.landau_tol), a.landau_maxit, eps, u, m[4]);
  const double g = rsqrt_nr(1.0 - u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
  const double n = g * (m[0] - u[0] * m[1] - u[1] * m[2] - u[2] * m[3]);
  const double T = eos_temperature_tab(tb, div_nr(eps, n), tb->c.zeta, flags);
  if (a.n) a.n[site] = n;
  if (a.eps) a.eps[site] = eps;
  if (a.T) a.T[site] = T;
  if (a.P) a.P[site] = n * T;
  if (a.ux) a.ux[site] = u[0];
  if (a.uy) a.uy[site] = u[1];
  if (uz) uz[site] = u[2];
  if (raw14)
    for (int k = 0; k < RLBM_NB3; ++k) raw14[k * S3 + site] = m[k];
}

// f_i(x, 0) = f_i^eq(n, T, u) on a 3D lattice
template <int P>
__global__ void __launch_bounds__(kBlock) k_init3(RlbmInitArgs a, const double* __restrict__ uz) {
  using S = typename Traits<P>::S;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long site = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (site >= (long long)L.nx * L.ny * L.nz) return;
  const int x = (int)(site % L.nx);
  const long long yz = site / L.nx;
  const int y = (int)(yz % L.ny), z = (int)(yz / L.ny);
  const double n = a.n[site], T = a.T[site];
  const double u[3] = {a.ux[site], a.uy[site], uz[site]};
  const double g = 1.0 / sqrt(1.0 - u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
  const double U[3] = {g * u[0], g * u[1], g * u[2]};
  double b[RLBM_NB3];
  projections3(proj_consts(tb), T, k1k2_ratio(tb->c.zeta / T), g, U, b);
  S* __restrict__ dst = (S*)a.dst;
  const long long o = (long long)(z + L.GZ) * L.zs + (long long)(y + L.GY) * L.rs + x + L.GX;
  for (int j = 0; j < tb->c.Q; ++j) {
    double fe = 0.0;
    for (int k = 0; k < RLBM_NB3; ++k) fe = fma(n * b[k] - (P == RLBM_FP64 ? 0.0 : tb->c.nb_ref3[k]), tb->row3d[j][k], fe);
    dst[(long long)j * L.cs + o] = to_store<P>((typename Traits<P>::A)fe, tb, j);
  }
}

// ------------------------------------------------------------------ moments

template <int P>
__global__ void __launch_bounds__(kBlock) k_moments(RlbmMomArgs a) {
  using S = typename Traits<P>::S;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long site = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (site >= (long long)L.nx * L.ny) return;
  const int y = (int)(site / L.nx), x = (int)(site - (long long)y * L.nx);
  const S* __restrict__ src = (const S*)a.src;
  double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < tb->c.Q; ++j) {
    const int sx = a.shift ? x - tb->nx[j] : x, sy = a.shift ? y - tb->ny[j] : y;
    const double f =
        (double)to_arith<P>(src[(long long)j * L.cs + (long long)(sy + L.GY) * L.rs + sx + L.GX], tb, j);
    const double p0 = tb->p0[j], px = tb->px[j], py = tb->py[j];
    m[0] += f * p0; m[1] += f * px; m[2] += f * py;
    m[3] += f * p0 * p0; m[4] += f * p0 * px; m[5] += f * p0 * py;
    m[6] += f * px * px; m[7] += f * px * py; m[8] += f * py * py;
  }
  if (P != RLBM_FP64)
    for (int k = 0; k < 9; ++k) m[k] += tb->c.ref_mom[k];
  Macro mac = macroscopic(tb, m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[8], a.landau_tol,
                          a.landau_maxit, a.landau_method);
  if (a.n) a.n[site] = mac.n;
  if (a.eps) a.eps[site] = mac.eps;
  if (a.T) a.T[site] = mac.T;
  if (a.P) a.P[site] = mac.P;
  if (a.ux) a.ux[site] = mac.ux;
  if (a.uy) a.uy[site] = mac.uy;
  if (a.raw9) {
    const long long S2 = (long long)L.nx * L.ny;
    for (int k = 0; k < 9; ++k) a.raw9[k * S2 + site] = m[k];
  }
}

// ------------------------------------------------------------------ init

template <int P>
__global__ void __launch_bounds__(kBlock) k_init(RlbmInitArgs a) {
  using S = typename Traits<P>::S;
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long site = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (site >= (long long)L.nx * L.ny) return;
  const int y = (int)(site / L.nx), x = (int)(site - (long long)y * L.nx);
  const double n = a.n[site], T = a.T[site], ux = a.ux[site], uy = a.uy[site];
  const double g = 1.0 / sqrt(1.0 - ux * ux - uy * uy);
  double b[RLBM_NB];
  projections(tb, T, k1k2_ratio(tb->c.zeta / T), g, g * ux, g * uy, b);
  double nb[RLBM_NB];
  for (int k = 0; k < RLBM_NB; ++k) nb[k] = n * b[k] - (P == RLBM_FP64 ? 0.0 : tb->c.nb_ref[k]);
  S* __restrict__ dst = (S*)a.dst;
  const long long o = (long long)(y + L.GY) * L.rs + x + L.GX;
  for (int j = 0; j < tb->c.Q; ++j) {
    double fe = 0.0;
    for (int k = 0; k < RLBM_NB; ++k) fe = fma(nb[k], tb->M[k][j], fe);
    dst[(long long)j * L.cs + o] = to_store<P>((typename Traits<P>::A)fe, tb, j);
  }
}

// ------------------------------------------------------------------ dispatch

using StepFn = void (*)(RlbmStepArgs);

// Class-count buckets: exact fits for the configured stencils (19: zeta = 1
// in 1D, 39: G1..G6 in 2D, 44: zeta = 1 in 2D, 73: the 133-population stencil
// in 2D) and padded buckets for any other stencil; the second argument is the
// bucket's smallest class count.
template <int P, bool G>
StepFn step_kernel(int Q) {
  if (Q <= 19) return k_step<19, 1, P, G>;
  if (Q <= 24) return k_step<24, 20, P, G>;
  if (Q <= 39) return k_step<39, 25, P, G>;
  if (Q <= 44) return k_step<44, 40, P, G>;
  if (Q <= 48) return k_step<48, 45, P, G>;
  if (Q <= 73) return k_step<73, 49, P, G>;
  if (Q <= 80) return k_step<80, 74, P, G>;
  return k_step<160, 81, P, G>;
}

// Generated fixed-stencil kernels, by id (see rlbm_fixed_stencils.h); with
// the learned guess for float32 storage only (nullptr otherwise).
template <class ST, int PREC>
StepFn fixed_kernel(bool guess) {
  if constexpr (PREC == RLBM_FP32_DEV) {
    if (guess) return k_step<ST::Q, ST::Q, PREC, true, ST>;
  } else {
    if (guess) return nullptr;
  }
  return k_step<ST::Q, ST::Q, PREC, false, ST>;
}

StepFn fixed_step(int id, bool guess) {
  switch (id) {
#define RLBM_FIXED_CASE(ID, ST, PREC) \
  case ID:                            \
    return fixed_kernel<rlbm_fixed::ST, PREC>(guess);
    RLBM_FIXED_KERNELS(RLBM_FIXED_CASE)
#undef RLBM_FIXED_CASE
    default:
      return nullptr;
  }
}

// The learned-guess kernels are built for float32 storage, the path the
// guess is meant for.
StepFn select_step(int prec, int Q, bool guess) {
  if (guess && prec == RLBM_FP32_DEV) return step_kernel<RLBM_FP32_DEV, true>(Q);
  switch (prec) {
    case RLBM_FP64: return step_kernel<RLBM_FP64, false>(Q);
    case RLBM_FP32_DEV: return step_kernel<RLBM_FP32_DEV, false>(Q);
    default: return step_kernel<RLBM_FP16_DEV, false>(Q);
  }
}

// 3D step kernels by class count (every population of the stencil is a class)
template <int P>
StepFn step3_kernel(int Q) {
  if (Q <= 48) return k_step3<48, 1, P>;
  if (Q <= 57) return k_step3<57, 49, P>;
  if (Q <= 73) return k_step3<73, 58, P>;
  if (Q <= 96) return k_step3<96, 74, P>;
  return k_step3<160, 97, P>;
}

StepFn select_step3(int prec, int Q) {
  switch (prec) {
    case RLBM_FP64: return step3_kernel<RLBM_FP64>(Q);
    case RLBM_FP32_DEV: return step3_kernel<RLBM_FP32_DEV>(Q);
    default: return step3_kernel<RLBM_FP16_DEV>(Q);
  }
}

// Generated third-order kernels, by id (see rlbm_fixed_stencils.h).
StepFn fixedo3_step(int id) {
  switch (id) {
#define RLBM_FIXEDO3_CASE(ID, ST, PREC, DIM) \
  case ID:                                  \
    return k_step_o3<DIM, PREC, rlbm_fixed::ST>;
    RLBM_FIXEDO3_KERNELS(RLBM_FIXEDO3_CASE)
#undef RLBM_FIXEDO3_CASE
    default:
      return nullptr;
  }
}

// Generated 3D kernels, by id (see rlbm_fixed_stencils.h).
StepFn fixed3_step(int id) {
  switch (id) {
#define RLBM_FIXED3_CASE(ID, ST, PREC) \
  case ID:                             \
    return k_step3<rlbm_fixed::ST::Q, rlbm_fixed::ST::Q, PREC, rlbm_fixed::ST>;
    RLBM_FIXED3_KERNELS(RLBM_FIXED3_CASE)
#undef RLBM_FIXED3_CASE
    default:
      return nullptr;
  }
}

// Diagnostic: the network's guess (eps, ux, uy) for the current state, from the
// same in-kernel inference as the step (one wave per 64 consecutive sites).
__global__ void __launch_bounds__(kBlock) k_guess(RlbmStepArgs a, float* __restrict__ out) {
  const TabPtr tb = as_tab(a.tab);
  const RlbmLayout& L = a.L;
  const long long S2 = (long long)L.nx * L.ny;
  const long long site0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long site = site0 < S2 ? site0 : S2 - 1;
  const int y = (int)(site / L.nx), x = (int)(site - (long long)y * L.nx);
  double md[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < tb->c.Q; ++j) {
    const int sx = a.shift ? x - tb->nx[j] : x, sy = a.shift ? y - tb->ny[j] : y;
    const long long idx = (long long)j * L.cs + (long long)(sy + L.GY) * L.rs + sx + L.GX;
    double f;
    if (tb->c.precision == RLBM_FP64) f = ((const double*)a.src)[idx];
    else if (tb->c.precision == RLBM_FP32_DEV) f = ((const float*)a.src)[idx];
    else f = (double)((float)((const _Float16*)a.src)[idx] * tb->scale[j]);
    const double p0 = tb->p0[j], px = tb->px[j], py = tb->py[j];
    md[0] += f * p0; md[1] += f * px; md[2] += f * py;
    md[3] += f * p0 * p0; md[4] += f * p0 * px; md[5] += f * p0 * py;
    md[6] += f * px * px; md[7] += f * px * py; md[8] += f * py * py;
  }
  if (tb->c.precision != RLBM_FP64)
    for (int k = 0; k < 9; ++k) md[k] += tb->c.ref_mom[k];
  float xin[9], yo[3];
  mlp_inputs(a, md, xin);
  mlp_wave(a, xin, yo);
  double e, ux, uy;
  mlp_destandardise(a, md[0], yo, e, ux, uy);
  if (site0 < S2) {
    out[site0] = (float)e;
    out[S2 + site0] = (float)ux;
    out[2 * S2 + site0] = (float)uy;
  }
}

size_t elem_size(int prec) { return prec == RLBM_FP64 ? 8 : prec == RLBM_FP32_DEV ? 4 : 2; }

}  // namespace rlbm

using namespace rlbm;

struct rlbm_ctx {
  RlbmTable* h_tab = nullptr;
  RlbmTable* d_tab = nullptr;
  rlbm_stencil_info info;
  int device = 0;
  bool have_fields = false;
  rlbm_lattice_desc lat;
  void* buf[2] = {nullptr, nullptr};
  size_t pop_bytes = 0;
  RlbmLayout L;
  int cur = 0;
  int shifted = 0;
  long long steps = 0;
  RlbmSlot* slots = nullptr;    // health slots in use: d_slots, or the static array
  RlbmSlot* d_slots = nullptr;  // library-allocated health slots
  int nslots = 0;               // capacity of d_slots
  bool static_slots = false;    // slots live in the device's static array
  int tiles_x = 0, ntiles = 0;  // wave tiles (kWave sites of a row); one health slot each
  double tk1 = 0, tk2 = 0;
  const rlbm_mlp* guess = nullptr;
  float* d_warm = nullptr;          // warm-start frames (3 planes of nx ny floats)
  size_t warm_cap = 0;              // floats allocated at d_warm
  bool warm = false;
  int fixed_id = -1;                // generated fixed-stencil kernel for this table, or -1
  int fixed3_id = -1;               // generated 3D kernel for this table, or -1
  int fixedo3_id = -1;              // generated third-order kernel for this table, or -1
  int variant = RLBM_STEP_AUTO;     // RLBM_STEP_AUTO or RLBM_STEP_TABLE
  char err[512] = {0};
};

static int fail(rlbm_ctx* c, int code, const char* fmt, const char* detail = "") {
  char msg[512];
  snprintf(msg, sizeof(msg), fmt, detail);
  if (c) snprintf(c->err, sizeof(c->err), "%s", msg);
  rlbm_set_global_error(msg);
  return code;
}

#define HIPCHECK(ctx, call)                                                  \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) return fail(ctx, RLBM_EHIP, "HIP error: %s", hipGetErrorString(e_)); \
  } while (0)

extern "C" int rlbm_init_stencil(rlbm_ctx** out, const rlbm_stencil_desc* desc, rlbm_stencil_info* info) {
  if (!out) return fail(nullptr, RLBM_EINVAL, "out is NULL");
  *out = nullptr;
  rlbm_ctx* c = new rlbm_ctx();
  c->h_tab = new RlbmTable();
  char err[512] = {0};
  int rc = rlbm_build_table(desc, &c->info, c->h_tab, err, sizeof(err));
  if (rc) {
    fail(nullptr, rc, "%s", err);
    delete c->h_tab;
    delete c;
    return rc;
  }
  rlbm_build_eos_table(desc->zeta, c->h_tab->eos);
  // a generated fixed-stencil kernel applies when this table is the one it was generated from
  c->fixed_id = -1;
  const uint64_t fp = rlbm_table_fingerprint(c->h_tab);
  for (int i = 0; i < rlbm_fixed::kNumFixed && c->h_tab->c.order == 2; ++i)
    if (rlbm_fixed::kFixedTables[i].fingerprint == fp && rlbm_fixed::kFixedTables[i].precision == c->h_tab->c.precision)
      c->fixed_id = i;
  c->fixed3_id = -1;
  for (int i = 0; i < rlbm_fixed::kNumFixed3 && c->h_tab->c.order == 2 && c->h_tab->c.dim == 3; ++i)
    if (rlbm_fixed::kFixed3Tables[i].fingerprint == fp &&
        rlbm_fixed::kFixed3Tables[i].precision == c->h_tab->c.precision)
      c->fixed3_id = i;
  c->fixedo3_id = -1;
  for (int i = 0; i < rlbm_fixed::kNumFixedO3 && c->h_tab->c.order == 3; ++i)
    if (rlbm_fixed::kFixedO3Tables[i].fingerprint == fp &&
        rlbm_fixed::kFixedO3Tables[i].precision == c->h_tab->c.precision &&
        rlbm_fixed::kFixedO3Tables[i].dim == c->h_tab->c.dim)
      c->fixedo3_id = i;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->d_tab, sizeof(RlbmTable));
  if (e == hipSuccess) e = hipMemcpy(c->d_tab, c->h_tab, sizeof(RlbmTable), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    fail(nullptr, RLBM_EHIP, "HIP error: %s", hipGetErrorString(e));
    if (c->d_tab) (void)hipFree(c->d_tab);
    delete c->h_tab;
    delete c;
    return RLBM_EHIP;
  }
  if (info) *info = c->info;
  *out = c;
  return RLBM_OK;
}

// ------------------------------------------------------------------ static health slots
//
// The allocation-free field set-up keeps the health slots of its lattice in
// one file-scope device array instead of library-allocated memory.  Each GPU
// holds its own copy of the array (until the process ends), found once per
// device with hipGetSymbolAddress; host code uses only that address, never
// the array's name.  One context per device owns it at a time: a context
// that takes it over drops the fields of the previous owner (whose later
// rlbm_step then returns RLBM_ESTATE), so no step of a context ever writes
// another lattice's slots.  Steps of the previous owner that are still in
// flight when the array changes hands write slots below that owner's tile
// count, which stays inside the array; only its health counters are mixed up
// (calls that overlap on one GPU race).
constexpr int kStaticSlots = 262144;  // 4 MiB: one slot per 64-site tile, e.g. a 4096 x 4096 lattice
static __device__ __align__(256) RlbmSlot scratch[kStaticSlots];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
RlbmSlot* g_static_ptr[kMaxDevices] = {};
rlbm_ctx* g_static_owner[kMaxDevices] = {};
}  // namespace

// Address of this device's static slot array (resolved once per device, with
// that device current); nullptr and *why on failure.
static RlbmSlot* static_slots_of(int device, const char** why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device index beyond the static-slot table";
    return nullptr;
  }
  if (!g_static_ptr[device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) {
      *why = "hipGetDevice failed";
      return nullptr;
    }
    if (prev != device && hipSetDevice(device) != hipSuccess) {
      *why = "hipSetDevice failed";
      return nullptr;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      *why = "hipGetSymbolAddress of the static slot array failed";
      return nullptr;
    }
    g_static_ptr[device] = (RlbmSlot*)p;
  }
  return g_static_ptr[device];
}

// Gives up c's claim on its device's static slot array (caller holds g_static_mu).
static void release_static_slots(rlbm_ctx* c) {
  if (c->device >= 0 && c->device < kMaxDevices && g_static_owner[c->device] == c) g_static_owner[c->device] = nullptr;
  if (c->static_slots) c->slots = nullptr;
  c->static_slots = false;
}

extern "C" int rlbm_destroy(rlbm_ctx* c) {
  if (!c) return RLBM_OK;
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    release_static_slots(c);
  }
  if (c->d_tab) (void)hipFree(c->d_tab);
  if (c->d_slots) (void)hipFree(c->d_slots);
  if (c->d_warm) (void)hipFree(c->d_warm);
  delete c->h_tab;
  delete c;
  return RLBM_OK;
}

// Row-interleaved layout: ghost columns padded to 32 elements so every
// interior class row starts on a 32-element boundary; ghost rows of the max
// |n_y|; the Q class rows of a lattice row are consecutive.
// 3D lattices stack nz + 2 GZ planes of storage rows (GZ = max |n_z|).
// Stencils whose lattices run on the 3D layout and entry points (3D
// stencils, and third-order stencils of every dimension).
static bool layout3(const RlbmConsts& k) { return k.dim == 3 || k.order == 3; }

static RlbmLayout make_layout(const RlbmConsts& k, int nx, int ny, int bc_x, int bc_y, int nz = 1, int bc_z = 0) {
  RlbmLayout L;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.Sx = k.sx_max;
  L.Sy = k.sy_max;
  L.Sz = k.dim == 3 ? k.sz_max : 0;
  L.GX = (L.Sx + 31) / 32 * 32;
  L.GY = L.Sy;
  L.GZ = L.Sz;
  L.W = (L.GX + nx + L.Sx + 31) / 32 * 32;
  L.cs = L.W;
  L.rs = (long long)k.Q * L.W;
  L.zs = (long long)(ny + 2 * L.GY) * L.rs;
  const long long s = (long long)(nz + 2 * L.GZ) * L.zs;
  L.total = (s + kPlaneAlign - 1) / kPlaneAlign * kPlaneAlign;
  L.bc_x = bc_x;
  L.bc_y = bc_y;
  L.bc_z = bc_z;
  return L;
}

extern "C" size_t rlbm_population_bytes(const rlbm_ctx* c, int nx, int ny) {
  if (!c || nx <= 0 || ny <= 0 || layout3(c->h_tab->c)) return 0;
  RlbmLayout L = make_layout(c->h_tab->c, nx, ny, 0, 0);
  return (size_t)L.total * elem_size(c->h_tab->c.precision);
}

extern "C" size_t rlbm_population_bytes3(const rlbm_ctx* c, int nx, int ny, int nz) {
  if (!c || nx <= 0 || ny <= 0 || nz <= 0 || !layout3(c->h_tab->c)) return 0;
  if (c->h_tab->c.dim != 3 && (nz != 1 || (c->h_tab->c.dim == 1 && ny != 1))) return 0;
  RlbmLayout L = make_layout(c->h_tab->c, nx, ny, 0, 0, nz, 0);
  return (size_t)L.total * elem_size(c->h_tab->c.precision);
}

// Everything about a lattice description that needs no device: sizes,
// boundary rules, relaxation time, Landau options, and the layout's limits
// (fewer than 2^31 stored elements, class byte offsets below 2^31).  Fills L
// and the class offsets (offs[0, QMAX): own storage, [QMAX, 2 QMAX): pulled).
// Returns nullptr, or the reason the description is rejected.
static const char* check_lattice(const RlbmTable& t, const rlbm_lattice_desc* lat, RlbmLayout& L,
                                 unsigned offs[2 * RLBM_QMAX]) {
  const RlbmConsts& k = t.c;
  if (!lat) return "NULL lattice description";
  const int nz = k.dim == 3 ? lat->nz : 1;
  if (lat->nx <= 0 || lat->ny <= 0 || (k.dim == 1 && lat->ny != 1))
    return "invalid lattice size (1D stencils need ny == 1)";
  if (k.dim == 3 ? lat->nz < 1 : (lat->nz < 0 || lat->nz > 1))
    return "invalid nz (>= 1 for 3D stencils, 0 or 1 otherwise)";
  if ((long long)lat->nx * lat->ny * nz > (1LL << 31) - 1) return "lattice too large";
  if (lat->bc_x < 0 || lat->bc_x > 1 || lat->bc_y < 0 || lat->bc_y > 1) return "invalid bc";
  if (k.dim == 3 && (lat->bc_z < 0 || lat->bc_z > 1)) return "invalid bc_z";
  if (layout3(k) && lat->landau_method != RLBM_LANDAU_NEWTON)
    return "3D and third-order lattices solve the Landau frame by Newton";
  if (lat->tau_mode == RLBM_TAU_CONST) {
    if (!(lat->tau > 0.5)) return "tau must exceed 1/2";
  } else if (lat->tau_mode == RLBM_TAU_ETA_OVER_S) {
    if (!(lat->eta_over_s > 0) || !(lat->T_R_GeV > 0) || !(lat->n_unit_fm3 > 0) || !(lat->dx_fm > 0))
      return "eta/s mode needs eta_over_s, T_R_GeV, n_unit_fm3, dx_fm > 0";
  } else {
    return "invalid tau mode";
  }
  if (lat->landau_maxit > 1000000) return "landau_maxit above 10^6";
  if (lat->landau_method != RLBM_LANDAU_NEWTON && lat->landau_method != RLBM_LANDAU_FIXED_POINT)
    return "invalid Landau method";
  L = make_layout(k, lat->nx, lat->ny, lat->bc_x, lat->bc_y, nz, k.dim == 3 ? lat->bc_z : 0);
  if (L.total >= (1LL << 31)) return "lattice too large (2^31 or more stored elements)";
  const long long es = (long long)elem_size(k.precision);
  const long long base = (long long)L.Sz * L.zs + (long long)L.Sy * L.rs + L.Sx;
  for (int j = 0; j < RLBM_QMAX; ++j) {
    const int jj = j < k.Q ? j : 0;  // padding classes read class 0's source
    const long long own = base + jj * L.cs;
    const long long src = own - (long long)t.nz[jj] * L.zs - (long long)t.ny[jj] * L.rs - t.nx[jj];
    if (src < 0 || es * (own + L.Sz * L.zs + L.Sy * L.rs + L.Sx + kWave) >= (1LL << 31))
      return "class offsets out of range";
    offs[j] = (unsigned)(es * own);
    offs[RLBM_QMAX + j] = (unsigned)(es * src);
  }
  return nullptr;
}

extern "C" int rlbm_check_lattice(const rlbm_stencil_desc* desc, const rlbm_lattice_desc* lat) {
  if (!desc || !lat) return fail(nullptr, RLBM_EINVAL, "NULL stencil or lattice description");
  std::unique_ptr<RlbmTable> t(new RlbmTable());
  rlbm_stencil_info info;
  char err[512] = {0};
  const int rc = rlbm_build_table(desc, &info, t.get(), err, sizeof(err));
  if (rc) return fail(nullptr, rc, "%s", err);
  RlbmLayout L;
  unsigned offs[2 * RLBM_QMAX];
  if (const char* why = check_lattice(*t, lat, L, offs)) return fail(nullptr, RLBM_EINVAL, "%s", why);
  return RLBM_OK;
}

// Device part of a field set-up: the class offsets of this lattice into the
// context's table, and cleared health slots (a fill kernel, so that the
// set-up records no memset node when a caller captures it in a graph).
struct RlbmOffsetsArg {
  unsigned v[2 * RLBM_QMAX];
};

__global__ void __launch_bounds__(kBlock) k_fields_setup(RlbmOffsetsArg o, RlbmTable* __restrict__ tab,
                                                         RlbmSlot* __restrict__ slots, int nslots) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < 2 * RLBM_QMAX; j += kBlock) tab->offs[j] = o.v[j];
  if (i < nslots) slots[i] = RlbmSlot{0u, 0u, 0ull};
}

// Shared body of rlbm_init_fields and rlbm_init_fields_noalloc.  With
// use_static the health slots live in the device's static array and nothing
// is allocated.
static int init_fields_impl(rlbm_ctx* c, const rlbm_lattice_desc* lat, const double* n, const double* T,
                            const double* ux, const double* uy, const double* uz, void* popA, void* popB,
                            size_t pop_bytes, void* stream, bool use_static, bool three_d) {
  if (!c || !lat) return fail(c, RLBM_EINVAL, "NULL context or lattice");
  const RlbmConsts& k = c->h_tab->c;
  if (layout3(k) != three_d)
    return fail(c, RLBM_EINVAL, "%s", three_d ? "rlbm_init_fields3 needs a 3D or third-order stencil"
                                              : "3D and third-order stencils take rlbm_init_fields3");
  RlbmLayout L;
  RlbmOffsetsArg offs;
  if (const char* why = check_lattice(*c->h_tab, lat, L, offs.v)) return fail(c, RLBM_EINVAL, "%s", why);
  if (!n || !T || !ux || !uy || (three_d && !uz) || !popA || !popB || popA == popB)
    return fail(c, RLBM_EINVAL, "NULL field or population buffer");
  const int nz = k.dim == 3 ? lat->nz : 1;
  const size_t need = three_d ? rlbm_population_bytes3(c, lat->nx, lat->ny, nz)
                              : rlbm_population_bytes(c, lat->nx, lat->ny);
  if (pop_bytes < need) return fail(c, RLBM_EINVAL, "population buffer too small");
  const int tiles_x = (lat->nx + kWave - 1) / kWave;
  const long long ntiles = (long long)tiles_x * lat->ny * nz;
  if (use_static && ntiles > kStaticSlots)
    return fail(c, RLBM_EINVAL, "%s",
                "lattice too large for the allocation-free set-up (more than 262144 tiles of 64 sites of a row)");
  hipStream_t s = (hipStream_t)stream;

  // from here on the context is being rebuilt: a failure leaves it without fields
  c->have_fields = false;
  RlbmSlot* slots = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (use_static) {
      const char* why = nullptr;
      slots = static_slots_of(c->device, &why);
      if (!slots) return fail(c, RLBM_EHIP, "%s", why);
      rlbm_ctx* prev = g_static_owner[c->device];
      if (prev && prev != c) {
        // the previous owner loses its fields (its slots are about to be reused)
        prev->have_fields = false;
        release_static_slots(prev);
        snprintf(prev->err, sizeof(prev->err), "%s",
                 "fields dropped: another context took the allocation-free health slots of this device");
      }
      g_static_owner[c->device] = c;
      c->static_slots = true;
    } else {
      release_static_slots(c);
    }
  }
  if (!use_static) {
    if (ntiles > c->nslots) {
      if (c->d_slots) HIPCHECK(c, hipFree(c->d_slots));
      c->d_slots = nullptr;
      c->nslots = 0;
      HIPCHECK(c, hipMalloc((void**)&c->d_slots, sizeof(RlbmSlot) * ntiles));
      c->nslots = (int)ntiles;
    }
    slots = c->d_slots;
  }
  c->slots = slots;
  c->lat = *lat;
  c->warm = false;
  if (!(c->lat.landau_tol > 0)) c->lat.landau_tol = k.precision == RLBM_FP64 ? 1e-14 : 1e-10;
  if (c->lat.landau_maxit <= 0) c->lat.landau_maxit = 200;
  c->buf[0] = popA;
  c->buf[1] = popB;
  c->pop_bytes = pop_bytes;
  c->L = L;
  c->cur = 0;
  c->shifted = 0;
  c->steps = 0;
  c->tiles_x = tiles_x;
  c->ntiles = (int)ntiles;
  if (lat->tau_mode == RLBM_TAU_ETA_OVER_S) {
    const double TR = lat->T_R_GeV;
    c->tk1 = 1.5 * lat->eta_over_s * kHbarC * k.v0 / (lat->dx_fm * TR);
    c->tk2 = lat->n_unit_fm3 * M_PI * M_PI * kHbarC * kHbarC * kHbarC / (16.0 * TR * TR * TR);
  }
  const long long nfill = std::max<long long>(ntiles, 1);
  hipLaunchKernelGGL(k_fields_setup, dim3((unsigned)((nfill + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, offs,
                     c->d_tab, slots, c->ntiles);
  HIPCHECK(c, hipGetLastError());
  RlbmInitArgs ia;
  ia.dst = popA;
  ia.L = c->L;
  ia.n = n; ia.T = T; ia.ux = ux; ia.uy = uy;
  ia.tab = c->d_tab;
  long long sites = (long long)lat->nx * lat->ny * nz;
  dim3 grid((unsigned)((sites + kBlock - 1) / kBlock));
  if (k.order == 3) {
    typedef void (*InitO3)(RlbmInitArgs, const double*);
    InitO3 ik;
    if (k.precision == RLBM_FP32_DEV)
      ik = k.dim == 1 ? k_init_o3<1, RLBM_FP32_DEV> : k.dim == 2 ? k_init_o3<2, RLBM_FP32_DEV> : k_init_o3<3, RLBM_FP32_DEV>;
    else
      ik = k.dim == 1 ? k_init_o3<1, RLBM_FP64> : k.dim == 2 ? k_init_o3<2, RLBM_FP64> : k_init_o3<3, RLBM_FP64>;
    hipLaunchKernelGGL(ik, grid, dim3(kBlock), 0, s, ia, uz);
  } else if (three_d) {
    switch (k.precision) {
      case RLBM_FP64: hipLaunchKernelGGL(k_init3<RLBM_FP64>, grid, dim3(kBlock), 0, s, ia, uz); break;
      case RLBM_FP32_DEV: hipLaunchKernelGGL(k_init3<RLBM_FP32_DEV>, grid, dim3(kBlock), 0, s, ia, uz); break;
      default: hipLaunchKernelGGL(k_init3<RLBM_FP16_DEV>, grid, dim3(kBlock), 0, s, ia, uz); break;
    }
  } else {
    switch (k.precision) {
      case RLBM_FP64: hipLaunchKernelGGL(k_init<RLBM_FP64>, grid, dim3(kBlock), 0, s, ia); break;
      case RLBM_FP32_DEV: hipLaunchKernelGGL(k_init<RLBM_FP32_DEV>, grid, dim3(kBlock), 0, s, ia); break;
      default: hipLaunchKernelGGL(k_init<RLBM_FP16_DEV>, grid, dim3(kBlock), 0, s, ia); break;
    }
  }
  HIPCHECK(c, hipGetLastError());
  c->have_fields = true;
  return RLBM_OK;
}

extern "C" int rlbm_init_fields(rlbm_ctx* c, const rlbm_lattice_desc* lat, const double* n, const double* T,
                                const double* ux, const double* uy, void* popA, void* popB, size_t pop_bytes,
                                void* stream) {
  return init_fields_impl(c, lat, n, T, ux, uy, nullptr, popA, popB, pop_bytes, stream, false, false);
}

extern "C" int rlbm_init_fields3(rlbm_ctx* c, const rlbm_lattice_desc* lat, const double* n, const double* T,
                                 const double* ux, const double* uy, const double* uz, void* popA, void* popB,
                                 size_t pop_bytes, void* stream) {
  return init_fields_impl(c, lat, n, T, ux, uy, uz, popA, popB, pop_bytes, stream, false, true);
}

extern "C" int rlbm_init_fields_noalloc(rlbm_ctx* c, const rlbm_lattice_desc* lat, const double* n,
                                        const double* T, const double* ux, const double* uy, void* popA,
                                        void* popB, size_t pop_bytes, void* stream) {
  return init_fields_impl(c, lat, n, T, ux, uy, nullptr, popA, popB, pop_bytes, stream, true, false);
}

extern "C" int rlbm_step(rlbm_ctx* c, int nsteps, void* stream) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_step before rlbm_init_fields");
  if (nsteps < 0) return fail(c, RLBM_EINVAL, "negative step count");
  hipStream_t s = (hipStream_t)stream;
  RlbmStepArgs a;
  a.L = c->L;
  a.tau_mode = c->lat.tau_mode;
  a.tau = c->lat.tau;
  a.inv_tau = 1.0 / c->lat.tau;
  a.tk1 = c->tk1;
  a.tk2 = c->tk2;
  a.landau_tol = c->lat.landau_tol;
  a.landau_maxit = c->lat.landau_maxit;
  a.landau_method = c->lat.landau_method;
  a.tab = c->d_tab;
  a.slots = c->slots;
  const bool g = c->guess != nullptr && c->h_tab->c.precision == RLBM_FP32_DEV;
  if (g) {
    a.mlp_frag = c->guess->frag;
    a.mlp_bias = c->guess->biasfrag;
    for (int i = 0; i < 24; ++i) a.mlp_norm[i] = c->guess->h_norm[i];
    for (int i = 0; i < 9; ++i) a.mlp_norm[9 + i] = 1.0f / c->guess->h_norm[9 + i];
  }
  const bool d3 = layout3(c->h_tab->c);
  StepFn fn = (!d3 && c->variant == RLBM_STEP_AUTO && c->fixed_id >= 0) ? fixed_step(c->fixed_id, g) : nullptr;
  if (!fn && d3 && c->variant == RLBM_STEP_AUTO && c->fixed3_id >= 0) fn = fixed3_step(c->fixed3_id);
  if (!fn && c->h_tab->c.order == 3 && c->variant == RLBM_STEP_AUTO && c->fixedo3_id >= 0)
    fn = fixedo3_step(c->fixedo3_id);
  if (!fn && c->h_tab->c.order == 3) {
    const int dim = c->h_tab->c.dim;
    if (c->h_tab->c.precision == RLBM_FP32_DEV)
      fn = dim == 1 ? k_step_o3<1, RLBM_FP32_DEV> : dim == 2 ? k_step_o3<2, RLBM_FP32_DEV> : k_step_o3<3, RLBM_FP32_DEV>;
    else
      fn = dim == 1 ? k_step_o3<1, RLBM_FP64> : dim == 2 ? k_step_o3<2, RLBM_FP64> : k_step_o3<3, RLBM_FP64>;
  }
  if (!fn) fn = d3 ? select_step3(c->h_tab->c.precision, c->h_tab->c.Q) : select_step(c->h_tab->c.precision, c->h_tab->c.Q, g);
  if (!fn) return fail(c, RLBM_ESTATE, "no step kernel for this stencil");
  a.tiles_x = c->tiles_x;
  a.ntiles = c->ntiles;
  // byte offsets as in the offset table (range-checked below 2^31 there)
  const long long es = c->h_tab->c.precision == RLBM_FP64 ? 8 : c->h_tab->c.precision == RLBM_FP32_DEV ? 4 : 2;
  a.fo_base = (unsigned)(es * ((long long)c->L.Sz * c->L.zs + (long long)c->L.Sy * c->L.rs + c->L.Sx));
  a.fo_cs = (unsigned)(es * c->L.cs);
  const unsigned nwg = (unsigned)((c->ntiles + kStepBlock / kWave - 1) / (kStepBlock / kWave));
  // class offsets of this lattice, in the context's device table
  const unsigned* d_offs = (const unsigned*)((const char*)c->d_tab + offsetof(RlbmTable, offs));
  for (int i = 0; i < nsteps; ++i) {
    a.src = c->buf[c->cur];
    a.dst = c->buf[1 - c->cur];
    a.shift = c->shifted;
    a.offs = d_offs + (c->shifted ? RLBM_QMAX : 0);
    a.offs_st = d_offs;
    a.warm = (c->warm && !g) ? c->d_warm : nullptr;
    a.warm_plane = (long long)c->L.nx * c->L.ny;
    a.fo_rs = c->shifted ? (int)(es * c->L.rs) : 0;
    a.fo_es = c->shifted ? (int)es : 0;
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(kStepBlock), 0, s, a);
    HIPCHECK(c, hipGetLastError());
    c->cur ^= 1;
    c->shifted = 1;
    c->steps++;
  }
  return RLBM_OK;
}

extern "C" int rlbm_moments3(rlbm_ctx* c, double* n, double* eps, double* T, double* P, double* ux, double* uy,
                             double* uz, double* raw14, void* stream) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (!layout3(c->h_tab->c)) return fail(c, RLBM_EINVAL, "rlbm_moments3 needs a 3D or third-order stencil");
  if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_moments3 before rlbm_init_fields3");
  RlbmMomArgs a;
  a.src = c->buf[c->cur];
  a.L = c->L;
  a.shift = c->shifted;
  a.landau_tol = c->lat.landau_tol;
  a.landau_maxit = c->lat.landau_maxit;
  a.landau_method = c->lat.landau_method;
  a.tab = c->d_tab;
  a.n = n; a.eps = eps; a.T = T; a.P = P; a.ux = ux; a.uy = uy; a.raw9 = nullptr;
  long long sites = (long long)a.L.nx * a.L.ny * a.L.nz;
  dim3 grid((unsigned)((sites + kBlock - 1) / kBlock));
  hipStream_t s = (hipStream_t)stream;
  switch (c->h_tab->c.precision) {
    case RLBM_FP64: hipLaunchKernelGGL(k_moments3<RLBM_FP64>, grid, dim3(kBlock), 0, s, a, uz, raw14); break;
    case RLBM_FP32_DEV: hipLaunchKernelGGL(k_moments3<RLBM_FP32_DEV>, grid, dim3(kBlock), 0, s, a, uz, raw14); break;
    default: hipLaunchKernelGGL(k_moments3<RLBM_FP16_DEV>, grid, dim3(kBlock), 0, s, a, uz, raw14); break;
  }
  HIPCHECK(c, hipGetLastError());
  return RLBM_OK;
}

extern "C" int rlbm_moments(rlbm_ctx* c, double* n, double* eps, double* T, double* P, double* ux, double* uy,
                            double* raw9, void* stream) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (layout3(c->h_tab->c)) return fail(c, RLBM_EINVAL, "3D and third-order stencils take rlbm_moments3");
  if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_moments before rlbm_init_fields");
  RlbmMomArgs a;
  a.src = c->buf[c->cur];
  a.L = c->L;
  a.shift = c->shifted;
  a.landau_tol = c->lat.landau_tol;
  a.landau_maxit = c->lat.landau_maxit;
  a.landau_method = c->lat.landau_method;
  a.tab = c->d_tab;
  a.n = n; a.eps = eps; a.T = T; a.P = P; a.ux = ux; a.uy = uy; a.raw9 = raw9;
  long long sites = (long long)a.L.nx * a.L.ny;
  dim3 grid((unsigned)((sites + kBlock - 1) / kBlock));
  hipStream_t s = (hipStream_t)stream;
  switch (c->h_tab->c.precision) {
    case RLBM_FP64: hipLaunchKernelGGL(k_moments<RLBM_FP64>, grid, dim3(kBlock), 0, s, a); break;
    case RLBM_FP32_DEV: hipLaunchKernelGGL(k_moments<RLBM_FP32_DEV>, grid, dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(k_moments<RLBM_FP16_DEV>, grid, dim3(kBlock), 0, s, a); break;
  }
  HIPCHECK(c, hipGetLastError());
  return RLBM_OK;
}

extern "C" int rlbm_get_health(rlbm_ctx* c, unsigned* flags, unsigned long long* iter_sum, unsigned* iter_max,
                               int reset, void* stream) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (!c->have_fields) return fail(c, RLBM_ESTATE, "no fields");
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(c, hipStreamSynchronize(s));
  std::vector<RlbmSlot> h(c->ntiles);
  HIPCHECK(c, hipMemcpy(h.data(), c->slots, sizeof(RlbmSlot) * c->ntiles, hipMemcpyDeviceToHost));
  unsigned f = 0, mx = 0;
  unsigned long long sm = 0;
  for (auto& x : h) {
    f |= x.flags;
    mx = mx > x.iter_max ? mx : x.iter_max;
    sm += x.iter_sum;
  }
  if (flags) *flags = f;
  if (iter_sum) *iter_sum = sm;
  if (iter_max) *iter_max = mx;
  if (reset) {
    HIPCHECK(c, hipMemsetAsync(c->slots, 0, sizeof(RlbmSlot) * c->ntiles, s));
    HIPCHECK(c, hipStreamSynchronize(s));
  }
  if (f & RLBM_H_FATAL) return fail(c, RLBM_ENUMERIC, "fatal health flag raised (0x%s)", "see flags");
  return RLBM_OK;
}

extern "C" long long rlbm_step_count(const rlbm_ctx* c) { return c ? c->steps : -1; }

extern "C" int rlbm_set_step_variant(rlbm_ctx* c, int variant) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (variant != RLBM_STEP_AUTO && variant != RLBM_STEP_TABLE) return fail(c, RLBM_EINVAL, "invalid step variant");
  c->variant = variant;
  return RLBM_OK;
}

extern "C" int rlbm_step_kernel(const rlbm_ctx* c) {
  if (!c) return RLBM_EINVAL;
  const bool g = c->guess != nullptr && c->h_tab->c.precision == RLBM_FP32_DEV;
  if (c->variant == RLBM_STEP_AUTO && layout3(c->h_tab->c))
    return (c->h_tab->c.order == 3 ? c->fixedo3_id : c->fixed3_id) >= 0 ? RLBM_STEP_FIXED : RLBM_STEP_TABLE;
  return (c->variant == RLBM_STEP_AUTO && c->fixed_id >= 0 && fixed_step(c->fixed_id, g)) ? RLBM_STEP_FIXED
                                                                                          : RLBM_STEP_TABLE;
}

extern "C" int rlbm_save_state(rlbm_ctx* c, void* dst, size_t bytes, long long* step, int* layout_flag,
                               void* stream) {
  if (!c || !dst || !c->have_fields) return fail(c, RLBM_EINVAL, "invalid save");
  if (bytes < c->pop_bytes) return fail(c, RLBM_EINVAL, "destination too small");
  HIPCHECK(c, hipMemcpyAsync(dst, c->buf[c->cur], c->pop_bytes, hipMemcpyDefault, (hipStream_t)stream));
  if (step) *step = c->steps;
  if (layout_flag) *layout_flag = c->shifted;
  return RLBM_OK;
}

extern "C" int rlbm_load_state(rlbm_ctx* c, const void* src, size_t bytes, long long step, int layout_flag,
                               void* stream) {
  if (!c || !src || !c->have_fields) return fail(c, RLBM_EINVAL, "invalid load");
  if (bytes < c->pop_bytes) return fail(c, RLBM_EINVAL, "source too small");
  HIPCHECK(c, hipMemcpyAsync(c->buf[c->cur], src, c->pop_bytes, hipMemcpyDefault, (hipStream_t)stream));
  c->steps = step;
  c->shifted = layout_flag ? 1 : 0;
  return RLBM_OK;
}

extern "C" const char* rlbm_last_error(const rlbm_ctx* c) { return c ? c->err : rlbm_global_error(); }

extern "C" int rlbm_set_landau_guess(rlbm_ctx* c, const rlbm_mlp* m) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (m && (c->h_tab->c.precision != RLBM_FP32_DEV || c->h_tab->c.dim == 3))
    return fail(c, RLBM_EINVAL, "the learned guess is available for float32 deviation storage in 1D and 2D");
  if (m && c->warm) return fail(c, RLBM_EINVAL, "the learned guess and the warm start are exclusive");
  c->guess = m;
  return RLBM_OK;
}

extern "C" int rlbm_set_warm_start(rlbm_ctx* c, int enable) {
  if (!c) return fail(nullptr, RLBM_EINVAL, "NULL context");
  if (!enable) {
    c->warm = false;
    return RLBM_OK;
  }
  if (!c->have_fields) return fail(c, RLBM_ESTATE, "rlbm_set_warm_start before rlbm_init_fields");
  if (c->guess) return fail(c, RLBM_EINVAL, "the learned guess and the warm start are exclusive");
  if (layout3(c->h_tab->c)) return fail(c, RLBM_EINVAL, "the warm start is available for second-order 1D and 2D stencils");
  const size_t need = (size_t)3 * c->L.nx * c->L.ny;
  if (c->warm_cap < need) {
    if (c->d_warm) HIPCHECK(c, hipFree(c->d_warm));
    c->d_warm = nullptr;
    c->warm_cap = 0;
    HIPCHECK(c, hipMalloc((void**)&c->d_warm, need * sizeof(float)));
    c->warm_cap = need;
  }
  // zero frames: the first step starts as without the warm start
  HIPCHECK(c, hipMemset(c->d_warm, 0, need * sizeof(float)));
  c->warm = true;
  return RLBM_OK;
}

extern "C" int rlbm_landau_guess_fields(rlbm_ctx* c, float* out, void* stream) {
  if (!c || !out) return fail(c, RLBM_EINVAL, "NULL argument");
  if (!c->have_fields || !c->guess) return fail(c, RLBM_ESTATE, "no fields or no network");
  RlbmStepArgs a;
  memset(&a, 0, sizeof(a));
  a.src = c->buf[c->cur];
  a.L = c->L;
  a.shift = c->shifted;
  a.tab = c->d_tab;
  a.mlp_frag = c->guess->frag;
  a.mlp_bias = c->guess->biasfrag;
  for (int i = 0; i < 24; ++i) a.mlp_norm[i] = c->guess->h_norm[i];
  for (int i = 0; i < 9; ++i) a.mlp_norm[9 + i] = 1.0f / c->guess->h_norm[9 + i];
  long long sites = (long long)c->L.nx * c->L.ny;
  hipLaunchKernelGGL(k_guess, dim3((unsigned)((sites + kBlock - 1) / kBlock)), dim3(kBlock), 0, (hipStream_t)stream,
                     a, out);
  HIPCHECK(c, hipGetLastError());
  return RLBM_OK;
}

// ====================================================================== copy ceiling
//
// A plain streaming copy (16-byte loads and stores, several in flight per
// lane, a grid of a few waves per SIMD striding over the buffer): the
// achievable HBM rate that the step kernels' traffic is compared with.

namespace rlbm {
constexpr int kCopyBlock = 256;
constexpr int kCopyUnroll = 4;

typedef unsigned U32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kCopyBlock) k_copy(U32x4* __restrict__ dst, const U32x4* __restrict__ src,
                                                     long long n16) {
  const long long stride = (long long)gridDim.x * kCopyBlock * kCopyUnroll;
  for (long long i = ((long long)blockIdx.x * kCopyBlock * kCopyUnroll) + threadIdx.x; i < n16; i += stride) {
    U32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const long long k = i + (long long)u * kCopyBlock;
      if (k < n16) v[u] = __builtin_nontemporal_load(src + k);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const long long k = i + (long long)u * kCopyBlock;
      if (k < n16) __builtin_nontemporal_store(v[u], dst + k);
    }
  }
}
}  // namespace rlbm

extern "C" int rlbm_device_copy(void* dst, const void* src, size_t bytes, int workgroups, void* stream) {
  if (!dst || !src || bytes % 16 != 0 || workgroups <= 0) {
    rlbm_set_global_error("rlbm_device_copy: NULL buffer, size not a multiple of 16 bytes or no workgroups");
    return RLBM_EINVAL;
  }
  if (bytes == 0) return RLBM_OK;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)workgroups), dim3(kCopyBlock), 0, (hipStream_t)stream, (U32x4*)dst,
                     (const U32x4*)src, (long long)(bytes / 16));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    rlbm_set_global_error(hipGetErrorString(e));
    return RLBM_EHIP;
  }
  return RLBM_OK;
}

// ====================================================================== batch
//
// Many independent 1D problems (float32 deviation storage, outflow ends, tau
// from eta/s), each with its own stencil, advanced for many steps in ONE
// cooperative launch that spans the whole chip: the sites of every problem
// are cut into tiles of 64 consecutive sites (one wave each, so a wave never
// straddles two problems and reads its stencil's rows through the scalar
// cache), the tiles are dealt round-robin to the waves of the grid, and a
// grid-wide barrier separates the steps.  Every wave takes part in every
// barrier, tiles or not, so the launch always drains.

namespace rlbm {

constexpr int kBatchBlock = 256;
constexpr int kBatchQ = 24;  // classes of a 1D stencil

struct RlbmBatchProblem {
  long long base;  // element offset of plane 0
  int W;           // plane length: L + 2 S, rounded up to 64
  int L, S;        // sites, ghost width (max |n_x|)
  int table;       // stencil index
  long long site_off;  // offset of the problem's sites in concatenated field arrays
  double tk1, tk2;     // tau = 1/2 + tk1 (4 - ln(tk2 n / T^3)) / T
};

struct RlbmBatchTile {
  int prob;         // problem index
  int x0;           // first site of the tile
  int left, right;  // neighbouring tiles of the same problem, -1 at its ends
};

// Batched tiles are dealt to the device's L2 domains (XCDs): every tile of a
// problem goes to one XCD, and each wave takes the tiles of the XCD it runs
// on.  kBatchXcds bins (the XCD count of the device); the wave's hardware XCC
// id picks its bin.
constexpr int kBatchXcds = 8;
constexpr int kSyncCount = 0;                  // [kBatchXcds] waves registered per bin
constexpr int kSyncMask = kBatchXcds;          // [kBatchXcds] XCC ids seen per bin (bit mask)
constexpr int kSyncAbort = 2 * kBatchXcds;     // set when a wave gives up
constexpr int kSyncDone = 2 * kBatchXcds + 1;  // [ntiles] steps completed per tile
constexpr unsigned kSpinLimit = 1u << 20;      // ~100 ms of polling per wait

struct BatchRow;

struct RlbmBatchArgs {
  const void* src;
  void* dst;
  int shift;
  int nsteps;
  int sample_every;
  float* samples;       // [nsamples][total_sites][12] or NULL
  long long total_sites;
  const RlbmBatchProblem* probs;
  const RlbmBatchTile* tiles;
  int ntiles;
  const RlbmTable* const* tables;
  const BatchRow* rows;  // [stencil][kBatchQ] packed 1D rows
  double landau_tol;
  int landau_maxit;
  RlbmSlot* slots;      // one per wave of the grid
  unsigned* sync;       // kSyncDone + ntiles words, zero at launch
  const int* xtiles;    // tile indices grouped by XCD bin
  int xoff[kBatchXcds + 1];
};

// Per-class coefficients of the 1D stencils, packed per stencil into one
// compact block (built on the host at batch creation) and read through scalar
// loads: a CU's waves step problems with different stencils, and the packed
// rows of several stencils fit the scalar cache together where the full
// tables do not.  A 1D class has p^y = 0, so the moment monomials odd in p^y
// or containing p^y p^y vanish (N^y, T^0y, T^xy, T^yy), u_y = 0, and the
// projections b_3, b_6, b_7, b_9 (odd in U_y or proportional to U_y^2)
// vanish with their reference values: only the terms below can be nonzero,
// so dropping the others changes no result.
constexpr int kBMom[5] = {0, 1, 3, 4, 6};      // N^0, N^x, T^00, T^0x, T^xx
constexpr int kBEq[6] = {0, 1, 2, 4, 5, 8};    // b_0, b_1, b_2, b_4, b_5, b_8
// 24 floats per class: moment rows (5) and n_x as float; their remainders (5)
// and n_x as int bits; equilibrium rows (6); their remainders (6)
constexpr int kBRow = 24;
struct alignas(16) BatchRow {
  float v[kBRow];
};
typedef const __attribute__((address_space(4))) BatchRow* BatchRowPtr;

// One site per lane of a 64-site tile of one problem: pull, moments (float32
// rows plus their rounding remainders), Landau frame, EOS, projections,
// equilibrium and relaxation, store, and the outflow ghosts at the problem's
// ends.  All lanes run: a lane past the end (act false) repeats the last site
// without storing, so the ghosts are written by one masked vector store per
// class (lanes 0..S-1) from the end site's value.
__device__ __forceinline__ void batch_site(const RlbmBatchArgs& a, const RlbmBatchProblem& pr, TabPtr tb, int Q,
                                           BatchRowPtr R, const float* __restrict__ src, float* __restrict__ dst,
                                           int x, int x0,
                                           bool act, int shift, float* __restrict__ sample, unsigned& flags,
                                           unsigned& iters) {
  const int lane = (int)threadIdx.x & (kWave - 1);
  const bool first = x0 == 0;                  // the tile holds site 0
  const bool last = x0 + kWave >= pr.L;        // the tile holds site L - 1
  const int lend = min(pr.L - 1 - x0, kWave - 1);
  float f[kBatchQ];
#pragma unroll
  for (int j = 0; j < kBatchQ; ++j) {
    const int nxj = j < Q ? __float_as_int(R[j].v[11]) : 0;
    f[j] = j < Q ? src[pr.base + (long long)j * pr.W + x + pr.S - (shift ? nxj : 0)] : 0.0f;
  }
  float m[5] = {0, 0, 0, 0, 0};
  float ml[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < kBatchQ; ++j) {
    if (j < Q) {
      const BatchRow r = load_row(R + j);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        m[k] = fmaf(f[j], r.v[k], m[k]);
        ml[k] = fmaf(f[j], r.v[6 + k], ml[k]);
      }
    }
  }
  double md[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) md[k] = tb->c.ref_mom[k];
#pragma unroll
  for (int k = 0; k < 5; ++k) md[kBMom[k]] += (double)m[k] + (double)ml[k];
  Macro mac = macroscopic(tb, md[0], md[1], md[2], md[3], md[4], md[5], md[6], md[7], md[8], a.landau_tol,
                          a.landau_maxit, RLBM_LANDAU_NEWTON);
  flags |= mac.flags;
  iters = (unsigned)mac.iters;
  if (sample) {
#pragma unroll
    for (int k = 0; k < 9; ++k) sample[k] = (float)md[k];
    sample[9] = (float)mac.eps;
    sample[10] = (float)mac.ux;
    sample[11] = (float)mac.uy;
  }
  const double tau = tau_eta_over_s(pr.tk1, pr.tk2, mac.n, mac.T);
  double b[RLBM_NB];
  projections(tb, mac.T, mac.R, mac.gamma, mac.gamma * mac.ux, mac.gamma * mac.uy, b);
  const double w0 = div_nr(mac.gamma, tau);
  const float W0 = (float)w0, WX = (float)(-w0 * tb->c.v0 * mac.ux);
  float nb[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) nb[k] = (float)(mac.n * b[kBEq[k]] - tb->c.nb_ref[kBEq[k]]);
#pragma unroll
  for (int j = 0; j < kBatchQ; ++j) {
    if (j < Q) {
      const BatchRow r = load_row(R + j);
      const float* e = r.v + 12;
      const float* el = r.v + 18;
      float feq = nb[0] * e[0], feql = nb[0] * el[0];
#pragma unroll
      for (int k = 1; k < 6; ++k) {
        feq = fmaf(nb[k], e[k], feq);
        feql = fmaf(nb[k], el[k], feql);
      }
      const float om = fmaf(WX, r.v[5], W0);
      const float out = fmaf(-om, (f[j] - feq) - feql, f[j]);
      float* q = dst + pr.base + (long long)j * pr.W + pr.S;
      if (act) q[x] = out;
      // outflow ghosts: the end sites stand for every site beyond them
      if (first) {
        const float v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, out), 0));
        if (lane < pr.S) q[-1 - lane] = v;
      }
      if (last) {
        const float v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, out), lend));
        if (lane < pr.S) q[pr.L + lane] = v;
      }
    }
  }
}

__device__ __forceinline__ unsigned sync_load(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane 0 polls until both neighbours have completed `need` steps (a missing
// neighbour counts as done); false when the wait was abandoned.
__device__ __forceinline__ bool wait_neighbours(const unsigned* sync, int left, int right, unsigned need) {
  const unsigned* done = sync + kSyncDone;
  int ok = 1;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    unsigned spins = 0;
    while ((left >= 0 && sync_load(done + left) < need) || (right >= 0 && sync_load(done + right) < need)) {
      if (++spins >= kSpinLimit || ((spins & 255u) == 0 && sync_load(sync + kSyncAbort) != 0)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  return __shfl(ok, 0) != 0;
}

__global__ void __launch_bounds__(kBatchBlock) k_batch(RlbmBatchArgs a) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int lane = (int)threadIdx.x & (kWave - 1);
  const int wave = (int)blockIdx.x * (kBatchBlock / kWave) + (int)(threadIdx.x >> 6);
  unsigned* sync = a.sync;
  // register with the L2 domain (XCD) this wave runs on
  const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20);  // HW_REG_XCC_ID, bits 3:0
  const int bin = (int)(xcc % kBatchXcds);
  int slot = 0;
  if (lane == 0) {
    slot = (int)__hip_atomic_fetch_add(sync + kSyncCount + bin, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_or(sync + kSyncMask + bin, 1u << (xcc & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  slot = __builtin_amdgcn_readfirstlane(__shfl(slot, 0));
  __threadfence();
  grid.sync();
  __threadfence();
  const int nw = (int)sync_load(sync + kSyncCount + bin);
  const unsigned seen = sync_load(sync + kSyncMask + bin);
  unsigned flags = 0, imax = 0, isum = 0;
  // two XCDs in one bin would split a problem over two L2s: refuse to run
  bool live = (seen & (seen - 1u)) == 0u;
  if (!live) flags |= RLBM_H_SYNC;
  // a bin that holds tiles but got no wave would leave its problems unstepped
  if (wave == 0)
    for (int x = 0; x < kBatchXcds; ++x)
      if (a.xoff[x + 1] > a.xoff[x] && sync_load(sync + kSyncCount + x) == 0u) flags |= RLBM_H_SYNC;
  const int* mine = a.xtiles + a.xoff[bin];
  const int nmine = a.xoff[bin + 1] - a.xoff[bin];
  const float* src = (const float*)a.src;
  float* dst = (float*)a.dst;
  int shift = a.shift;
  for (int t = 0; t < a.nsteps && live; ++t) {
    const bool sampling = a.samples != nullptr && (t % a.sample_every) == 0;
    for (int k = slot; k < nmine && live; k += nw) {
      const int tile = mine[k];
      const RlbmBatchTile tl = a.tiles[tile];
      // the neighbours' step t - 1 stores sit in this XCD's L2; drop this
      // CU's L1 copies before pulling across the tile's edges
      if (t > 0 && !wait_neighbours(sync, tl.left, tl.right, (unsigned)t)) {
        live = false;
        flags |= RLBM_H_SYNC;
        if (lane == 0) __hip_atomic_store(sync + kSyncAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      asm volatile("buffer_inv sc0" ::: "memory");
      const int prob = __builtin_amdgcn_readfirstlane(tl.prob);
      const RlbmBatchProblem pr = a.probs[prob];
      const TabPtr tb = as_tab(a.tables[pr.table]);
      const int Q = tb->c.Q;
      const int x0 = __builtin_amdgcn_readfirstlane(tl.x0);
      const int x = x0 + lane;
      const bool act = x < pr.L;
      {
        float* srow = sampling && act
                          ? a.samples + ((long long)(t / a.sample_every) * a.total_sites + pr.site_off + x) * 12
                          : nullptr;
        unsigned it = 0, fl = 0;
        batch_site(a, pr, tb, Q, (BatchRowPtr)(a.rows + (long long)pr.table * kBatchQ), src, dst,
                   act ? x : pr.L - 1, x0, act, shift, srow, fl, it);
        if (act) {
          flags |= fl;
          imax = max(imax, it);
          isum += it;
        }
      }
      // this wave's stores have reached the XCD's L2 before the tile is
      // marked done (the L1 writes through)
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (lane == 0)
        __hip_atomic_store(sync + kSyncDone + tile, (unsigned)(t + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const float* tmp = src;
    src = dst;
    dst = (float*)tmp;
    shift = 1;
  }
  // per-wave statistics into the wave's own slot
  wave_stats(a.slots, wave, flags, imax, isum);
}

__global__ void __launch_bounds__(256) k_fill_u32(unsigned* __restrict__ p, long long n, unsigned v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// f = f^eq(n, T, u) of every problem (fields concatenated over the problems)
__global__ void __launch_bounds__(256) k_batch_init(const RlbmBatchProblem* probs, const RlbmTable* const* tables,
                                                  const double* __restrict__ n, const double* __restrict__ T,
                                                  const double* __restrict__ ux, float* __restrict__ dst) {
  const RlbmBatchProblem pr = probs[blockIdx.x];
  const TabPtr tb = as_tab(tables[pr.table]);
  for (int x = threadIdx.x; x < pr.L; x += 256) {
    const long long i = pr.site_off + x;
    const double u = ux[i];
    const double g = 1.0 / sqrt(1.0 - u * u);
    double b[RLBM_NB];
    projections(tb, T[i], k1k2_ratio(tb->c.zeta / T[i]), g, g * u, 0.0, b);
    for (int j = 0; j < tb->c.Q; ++j) {
      double fe = 0.0;
      for (int k = 0; k < RLBM_NB; ++k) fe = fma(n[i] * b[k] - tb->c.nb_ref[k], tb->M[k][j], fe);
      dst[pr.base + (long long)j * pr.W + pr.S + x] = (float)fe;
    }
  }
}

// pre-collision fields of every problem
__global__ void __launch_bounds__(256) k_batch_moments(const RlbmBatchProblem* probs, const RlbmTable* const* tables,
                                                     const float* __restrict__ src, int shift, double tol, int maxit,
                                                     double* n, double* eps, double* T, double* P, double* ux) {
  const RlbmBatchProblem pr = probs[blockIdx.x];
  const TabPtr tb = as_tab(tables[pr.table]);
  for (int x = threadIdx.x; x < pr.L; x += 256) {
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < tb->c.Q; ++j) {
      const double f = src[pr.base + (long long)j * pr.W + x + pr.S - (shift ? tb->nx[j] : 0)];
      const double p0 = tb->p0[j], px = tb->px[j];
      m[0] += f * p0; m[1] += f * px; m[3] += f * p0 * p0; m[4] += f * p0 * px; m[6] += f * px * px;
    }
    for (int k = 0; k < 9; ++k) m[k] += tb->c.ref_mom[k];
    Macro mac = macroscopic(tb, m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[8], tol, maxit,
                            RLBM_LANDAU_NEWTON);
    const long long i = pr.site_off + x;
    if (n) n[i] = mac.n;
    if (eps) eps[i] = mac.eps;
    if (T) T[i] = mac.T;
    if (P) P[i] = mac.P;
    if (ux) ux[i] = mac.ux;
  }
}

}  // namespace rlbm

struct rlbm_batch {
  int nprob = 0;
  std::vector<RlbmBatchProblem> h_probs;
  RlbmBatchProblem* d_probs = nullptr;
  const RlbmTable** d_tables = nullptr;
  BatchRow* d_rows = nullptr;        // [stencil][kBatchQ] packed 1D rows
  long long total_sites = 0, total_elems = 0;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0, shifted = 0;
  long long steps = 0;
  bool have_fields = false;
  RlbmSlot* d_slots = nullptr;      // one per wave of the cooperative grid
  RlbmBatchTile* d_tiles = nullptr;  // 64-site tiles of every problem
  int ntiles = 0;
  int* d_xtiles = nullptr;           // tile indices grouped by XCD bin
  int xoff[kBatchXcds + 1] = {};
  unsigned* d_sync = nullptr;        // per-launch hand-over state (kSyncDone + ntiles words)
  int workgroups = 0;                // cooperative grid (kBatchBlock threads each)
  int resident_limit = 0;            // workgroups the device holds at once for k_batch
  double landau_tol = 1e-10;
  int landau_maxit = 200;
};

static int bfail(const char* msg) {
  rlbm_set_global_error(msg);
  return RLBM_EINVAL;
}

#define BHIP(call)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      char b_[256];                                                                    \
      snprintf(b_, sizeof(b_), "HIP error: %s", hipGetErrorString(e_));                \
      rlbm_set_global_error(b_);                                                       \
      return RLBM_EHIP;                                                                \
    }                                                                                  \
  } while (0)

extern "C" int rlbm_batch_create(rlbm_batch** out, int nstencils, rlbm_ctx* const* stencils, int nprob,
                                 const rlbm_problem* probs, double landau_tol, int landau_maxit) {
  if (!out || nstencils <= 0 || !stencils || nprob <= 0 || !probs) return bfail("rlbm_batch_create: invalid argument");
  *out = nullptr;
  for (int s = 0; s < nstencils; ++s) {
    const RlbmConsts& k = stencils[s]->h_tab->c;
    if (k.dim != 1 || k.precision != RLBM_FP32_DEV || k.Q > kBatchQ)
      return bfail("rlbm_batch_create: stencils must be 1D, float32 deviation, at most 24 classes");
  }
  rlbm_batch* b = new rlbm_batch();
  b->nprob = nprob;
  b->landau_tol = landau_tol > 0 ? landau_tol : 1e-10;
  b->landau_maxit = landau_maxit > 0 ? landau_maxit : 200;
  long long elems = 0, sites = 0;
  for (int p = 0; p < nprob; ++p) {
    const rlbm_problem& q = probs[p];
    if (q.nx <= 0 || q.stencil < 0 || q.stencil >= nstencils || !(q.eta_over_s > 0) || !(q.T_R_GeV > 0) ||
        !(q.n_unit_fm3 > 0) || !(q.dx_fm > 0)) {
      delete b;
      return bfail("rlbm_batch_create: invalid problem");
    }
    const rlbm_ctx* c = stencils[q.stencil];
    const RlbmConsts& k = c->h_tab->c;
    RlbmBatchProblem pr;
    pr.S = k.sx_max;
    pr.L = q.nx;
    pr.W = (q.nx + 2 * pr.S + 63) / 64 * 64;
    pr.base = elems;
    pr.table = q.stencil;
    pr.site_off = sites;
    pr.tk1 = 1.5 * q.eta_over_s * kHbarC * k.v0 / (q.dx_fm * q.T_R_GeV);
    pr.tk2 = q.n_unit_fm3 * M_PI * M_PI * kHbarC * kHbarC * kHbarC / (16.0 * q.T_R_GeV * q.T_R_GeV * q.T_R_GeV);
    elems += (long long)k.Q * pr.W;
    sites += q.nx;
    b->h_probs.push_back(pr);
  }
  b->total_sites = sites;
  b->total_elems = elems;
  // 64-site tiles of every problem; whole problems are dealt to the XCD bins
  // (largest first, each to the bin with the fewest tiles so far)
  std::vector<RlbmBatchTile> tiles;
  std::vector<int> first(nprob), count(nprob);
  for (int p = 0; p < nprob; ++p) {
    first[p] = (int)tiles.size();
    for (int x0 = 0; x0 < b->h_probs[p].L; x0 += kWave) {
      const int i = (int)tiles.size();
      const bool last = x0 + kWave >= b->h_probs[p].L;
      tiles.push_back(RlbmBatchTile{p, x0, x0 == 0 ? -1 : i - 1, last ? -1 : i + 1});
    }
    count[p] = (int)tiles.size() - first[p];
  }
  b->ntiles = (int)tiles.size();
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return count[u] > count[v]; });
  std::vector<std::vector<int>> bins(kBatchXcds);
  std::vector<long long> load(kBatchXcds, 0);
  for (int p : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (int i = 0; i < count[p]; ++i) bins[x].push_back(first[p] + i);
    load[x] += count[p];
  }
  std::vector<int> xtiles;
  for (int x = 0; x < kBatchXcds; ++x) {
    b->xoff[x] = (int)xtiles.size();
    xtiles.insert(xtiles.end(), bins[x].begin(), bins[x].end());
  }
  b->xoff[kBatchXcds] = (int)xtiles.size();
  // the cooperative grid: one wave per tile, no more workgroups than the
  // device holds at once (a cooperative launch needs them all resident)
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, kBatchBlock, 0) != hipSuccess || per_cu < 1) {
    delete b;
    return bfail("rlbm_batch_create: occupancy query failed");
  }
  b->resident_limit = per_cu * cus;
  // waves are spread evenly over the XCDs, so size the grid for the fullest
  // bin: one wave per tile there
  long long fullest = 0;
  for (int x = 0; x < kBatchXcds; ++x) fullest = std::max<long long>(fullest, b->xoff[x + 1] - b->xoff[x]);
  const int want = (int)((fullest * kBatchXcds + kBatchBlock / kWave - 1) / (kBatchBlock / kWave));
  b->workgroups = std::max(1, std::min(want, b->resident_limit));
  const int nwaves = b->workgroups * (kBatchBlock / kWave);
  std::vector<const RlbmTable*> tabs(nstencils);
  for (int s = 0; s < nstencils; ++s) tabs[s] = stencils[s]->d_tab;
  // packed 1D rows of every stencil (layout of BatchRow)
  std::vector<BatchRow> rows((size_t)nstencils * kBatchQ);
  for (int s = 0; s < nstencils; ++s) {
    const RlbmTable& t = *stencils[s]->h_tab;
    for (int j = 0; j < t.c.Q; ++j) {
      float* r = rows[(size_t)s * kBatchQ + j].v;
      for (int k = 0; k < 5; ++k) {
        r[k] = t.rowmf[j][kBMom[k]];
        r[6 + k] = t.rowmf_lo[j][kBMom[k]];
      }
      r[5] = t.rowf[j][RLBM_R_NX];
      int nx = t.nx[j];
      memcpy(&r[11], &nx, sizeof(nx));
      for (int k = 0; k < 6; ++k) {
        r[12 + k] = t.rowf[j][kBEq[k]];
        r[18 + k] = t.rowf_lo[j][kBEq[k]];
      }
    }
  }
  if (hipMalloc((void**)&b->d_probs, sizeof(RlbmBatchProblem) * nprob) != hipSuccess ||
      hipMalloc((void**)&b->d_tables, sizeof(RlbmTable*) * nstencils) != hipSuccess ||
      hipMalloc((void**)&b->d_rows, sizeof(BatchRow) * rows.size()) != hipSuccess ||
      hipMalloc((void**)&b->d_slots, sizeof(RlbmSlot) * nwaves) != hipSuccess ||
      hipMalloc((void**)&b->d_tiles, sizeof(RlbmBatchTile) * b->ntiles) != hipSuccess ||
      hipMalloc((void**)&b->d_xtiles, sizeof(int) * b->ntiles) != hipSuccess ||
      hipMalloc((void**)&b->d_sync, sizeof(unsigned) * (kSyncDone + b->ntiles)) != hipSuccess) {
    rlbm_batch_destroy(b);
    return bfail("rlbm_batch_create: device allocation failed");
  }
  BHIP(hipMemcpy(b->d_probs, b->h_probs.data(), sizeof(RlbmBatchProblem) * nprob, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_tables, tabs.data(), sizeof(RlbmTable*) * nstencils, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_rows, rows.data(), sizeof(BatchRow) * rows.size(), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_tiles, tiles.data(), sizeof(RlbmBatchTile) * b->ntiles, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_xtiles, xtiles.data(), sizeof(int) * b->ntiles, hipMemcpyHostToDevice));
  BHIP(hipMemset(b->d_slots, 0, sizeof(RlbmSlot) * nwaves));
  *out = b;
  return RLBM_OK;
}

extern "C" int rlbm_batch_occupancy(const rlbm_batch* b, int* workgroups, int* resident_limit, int* tiles) {
  if (!b) return bfail("rlbm_batch_occupancy: NULL");
  if (workgroups) *workgroups = b->workgroups;
  if (resident_limit) *resident_limit = b->resident_limit;
  if (tiles) *tiles = b->ntiles;
  return RLBM_OK;
}

extern "C" int rlbm_batch_destroy(rlbm_batch* b) {
  if (!b) return RLBM_OK;
  (void)hipDeviceSynchronize();
  if (b->d_probs) (void)hipFree(b->d_probs);
  if (b->d_tables) (void)hipFree((void*)b->d_tables);
  if (b->d_rows) (void)hipFree(b->d_rows);
  if (b->d_slots) (void)hipFree(b->d_slots);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_xtiles) (void)hipFree(b->d_xtiles);
  if (b->d_sync) (void)hipFree(b->d_sync);
  delete b;
  return RLBM_OK;
}

extern "C" size_t rlbm_batch_population_bytes(const rlbm_batch* b) {
  return b ? (size_t)b->total_elems * sizeof(float) : 0;
}

extern "C" long long rlbm_batch_sites(const rlbm_batch* b) { return b ? b->total_sites : -1; }

extern "C" int rlbm_batch_init(rlbm_batch* b, const double* n, const double* T, const double* ux, void* popA,
                               void* popB, size_t bytes, void* stream) {
  if (!b || !n || !T || !ux || !popA || !popB || popA == popB) return bfail("rlbm_batch_init: invalid argument");
  if (bytes < rlbm_batch_population_bytes(b)) return bfail("rlbm_batch_init: buffers too small");
  b->buf[0] = popA;
  b->buf[1] = popB;
  b->cur = 0;
  b->shifted = 0;
  b->steps = 0;
  hipStream_t s = (hipStream_t)stream;
  BHIP(hipMemsetAsync(b->d_slots, 0, sizeof(RlbmSlot) * b->workgroups * (kBatchBlock / kWave), s));
  hipLaunchKernelGGL(k_batch_init, dim3(b->nprob), dim3(256), 0, s, b->d_probs, b->d_tables, n, T, ux,
                     (float*)popA);
  BHIP(hipGetLastError());
  b->have_fields = true;
  return RLBM_OK;
}

extern "C" int rlbm_batch_step_persistent(rlbm_batch* b, int nsteps, int sample_every, float* samples, void* stream) {
  if (!b || !b->have_fields) return bfail("rlbm_batch_step_persistent: no fields");
  if (nsteps < 0 || (samples && sample_every <= 0)) return bfail("rlbm_batch_step_persistent: invalid argument");
  if (nsteps == 0) return RLBM_OK;
  RlbmBatchArgs a;
  a.src = b->buf[b->cur];
  a.dst = b->buf[1 - b->cur];
  a.shift = b->shifted;
  a.nsteps = nsteps;
  a.sample_every = sample_every > 0 ? sample_every : 1;
  a.samples = samples;
  a.total_sites = b->total_sites;
  a.probs = b->d_probs;
  a.tables = b->d_tables;
  a.rows = b->d_rows;
  a.landau_tol = b->landau_tol;
  a.landau_maxit = b->landau_maxit;
  a.slots = b->d_slots;
  a.tiles = b->d_tiles;
  a.ntiles = b->ntiles;
  a.sync = b->d_sync;
  a.xtiles = b->d_xtiles;
  for (int x = 0; x <= kBatchXcds; ++x) a.xoff[x] = b->xoff[x];
  const long long nsync = kSyncDone + b->ntiles;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<long long>((nsync + 255) / 256, 1024)), dim3(256), 0,
                     (hipStream_t)stream, b->d_sync, nsync, 0u);
  BHIP(hipGetLastError());
  void* kargs[] = {&a};
  BHIP(hipLaunchCooperativeKernel((const void*)k_batch, dim3(b->workgroups), dim3(kBatchBlock), kargs, 0,
                                  (hipStream_t)stream));
  BHIP(hipGetLastError());
  if (nsteps % 2) b->cur ^= 1;
  b->shifted = 1;
  b->steps += nsteps;
  return RLBM_OK;
}

extern "C" int rlbm_batch_moments(rlbm_batch* b, double* n, double* eps, double* T, double* P, double* ux,
                                  void* stream) {
  if (!b || !b->have_fields) return bfail("rlbm_batch_moments: no fields");
  hipLaunchKernelGGL(k_batch_moments, dim3(b->nprob), dim3(256), 0, (hipStream_t)stream, b->d_probs, b->d_tables,
                     (const float*)b->buf[b->cur], b->shifted, b->landau_tol, b->landau_maxit, n, eps, T, P, ux);
  BHIP(hipGetLastError());
  return RLBM_OK;
}

extern "C" int rlbm_batch_get_health(rlbm_batch* b, unsigned* flags, unsigned long long* iter_sum,
                                     unsigned* iter_max, void* stream) {
  if (!b) return bfail("rlbm_batch_get_health: NULL");
  BHIP(hipStreamSynchronize((hipStream_t)stream));
  const int nslots = b->workgroups * (kBatchBlock / kWave);
  std::vector<RlbmSlot> h(nslots);
  BHIP(hipMemcpy(h.data(), b->d_slots, sizeof(RlbmSlot) * nslots, hipMemcpyDeviceToHost));
  unsigned f = 0, mx = 0;
  unsigned long long sm = 0;
  for (auto& x : h) {
    f |= x.flags;
    mx = mx > x.iter_max ? mx : x.iter_max;
    sm += x.iter_sum;
  }
  if (flags) *flags = f;
  if (iter_sum) *iter_sum = sm;
  if (iter_max) *iter_max = mx;
  return (f & RLBM_H_FATAL) ? RLBM_ENUMERIC : RLBM_OK;
}
