// Device side of libdg2p: HIP kernels for gfx950 (wave64).
//
// Mapping: one lane per GLL node.  An element of 4^d nodes occupies 4^d
// consecutive lanes (1D: 4 lanes, 16 elements per wave; 2D: 16 lanes, 4
// elements per wave; 3D: the whole wave), so a wave-wide load of one field
// of U[f][e][j] is 512 contiguous bytes.  The lane index inside an element is
// the node index j = a_x + 4 a_y + 16 a_z: the nodes of an x-line form a quad
// of lanes, those of a y-line sit at stride 4 inside a 16-lane row and those
// of a z-line at stride 16.  The 4-point derivative contraction along x uses
// DPP quad rotations, along y DPP row rotations (both plain VALU moves, no LDS
// traffic) and along z cross-row lane swaps; the per-lane coefficients are the
// rows of D rotated to match the lane each moved value comes from.
//
// Workgroups are 4 independent waves (256 threads).  Consecutive workgroups
// are dispatched round-robin over the 8 XCDs; the kernels remap the
// workgroup index so that each XCD sweeps one contiguous slab of elements,
// which keeps face neighbours in the same L2.
//
// Every element evaluates all of its own faces ("owner computes"): the
// numerical fluxes are recomputed from both traces by the two elements that
// share a face, so no face value is written twice and results are
// deterministic without atomics.  The neighbour's normal interface flux
// a.e_k and viscous traction tau.e_k at its face nodes need its own
// element-local gradients; they come from a face-ingredient buffer G that is
// written by the epilogue of the pass producing that state (the previous RK
// stage, or an ingredient pass for the first stage).  The same epilogue emits
// per-workgroup reduction records (largest wave speed, largest kinematic
// viscosity, alpha range, non-physical count, field integrals, deviations
// from reference P and u) from which the next time step and the monitors are
// reduced in a fixed order.

#pragma once

#include <hip/hip_runtime.h>

#include "../../include/dg2p.h"

namespace dg2p {

constexpr int BLOCK = 256;      // threads per workgroup (4 independent waves)
// Threads per workgroup of the element passes: hexahedra run one wave (one
// element) per workgroup, so that a finished wave's slot takes new work at
// once instead of waiting for the other waves of a four-wave workgroup; the
// other dimensions keep four waves (their small grids reduce the time step
// inside the first stage, which needs the records of few workgroups).
template <int DIM>
constexpr int ewg() {
  return DIM == 3 ? 64 : BLOCK;
}
// minimum resident waves per SIMD the register allocator targets, per dimension
#ifndef DG2P_WAVES_1D
#define DG2P_WAVES_1D 4
#endif
#ifndef DG2P_WAVES_2D
#define DG2P_WAVES_2D 3
#endif
// hexahedra: two waves (at most 256 VGPRs; their kernels use 194-256, none
// spills), declared so that the allocator cannot drift to one wave
#ifndef DG2P_WAVES_3D
#define DG2P_WAVES_3D 2
#endif
// Ends a value's code motion at this point (an empty asm statement that
// takes and returns the value in a vector register).
#ifndef DG2P_PIN
#define DG2P_PIN(x) asm volatile("" : "+v"(x))
#endif
// the viscous quad kernel (velocity gradient and tractions on top) runs two
// waves per SIMD: within three waves' registers it spills
#ifndef DG2P_WAVES_2D_VISC
#define DG2P_WAVES_2D_VISC 2
#endif
template <int DIM, bool VISC = false>
constexpr int min_waves() {
  return DIM == 1 ? DG2P_WAVES_1D : (DIM == 2 ? (VISC ? DG2P_WAVES_2D_VISC : DG2P_WAVES_2D) : DG2P_WAVES_3D);
}
constexpr int REC = 16;         // doubles per reduction record
// record slots
constexpr int R_WAVE = 0, R_NU = 1, R_AMIN = 2, R_AMAX = 3, R_BAD = 4, R_DEVP = 5, R_DEVU = 6,
              R_INT = 7;        // R_INT .. R_INT+7: field integrals

// ---- GLL tables of degree 3, built at compile time ----------------------------
// Nodes -1, -1/sqrt(5), 1/sqrt(5), 1; weights 1/6, 5/6, 5/6, 1/6;
// D[a][b] = l_b'(x_a) from the product rule of the Lagrange basis.
constexpr double csqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
  return r;
}
constexpr double GLL_S = 1.0 / csqrt(5.0);
struct GllTab {
  double x[4], w[4], D[4][4];
};
constexpr GllTab make_gll() {
  GllTab t{};
  t.x[0] = -1.0;
  t.x[1] = -GLL_S;
  t.x[2] = GLL_S;
  t.x[3] = 1.0;
  t.w[0] = t.w[3] = 1.0 / 6.0;
  t.w[1] = t.w[2] = 5.0 / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      if (a == b) {
        double s = 0.0;
        for (int m = 0; m < 4; ++m)
          if (m != a) s += 1.0 / (t.x[a] - t.x[m]);
        t.D[a][b] = s;
      } else {
        double num = 1.0, den = 1.0;
        for (int m = 0; m < 4; ++m) {
          if (m != b) den *= (t.x[b] - t.x[m]);
          if (m != a && m != b) num *= (t.x[a] - t.x[m]);
        }
        t.D[a][b] = num / den;
      }
    }
  return t;
}
constexpr GllTab GLL = make_gll();
// rotated coefficient tables: x quad rotation r, y row rotation by 4r, z lane xor 16r
constexpr double CX(int a, int r) { return GLL.D[a][(a + r) & 3]; }
constexpr double CY(int a, int r) { return GLL.D[a][(a - r) & 3]; }
constexpr double CZ(int a, int r) { return GLL.D[a][a ^ r]; }

// The same coefficients as a table read with the lane's own a_k (a load from
// cached constant memory instead of a selection among compile-time
// constants, which compiles to branches): c[k][a][r] = the axis-k rotation
// r coefficient of a node at position a; sp[0][a] = D[0][a] / w_a and
// sp[1][a] = D[3][a] / w_a, the SIPG spread weights of the line's low and
// high ends; w[a] the GLL weight.
struct CoefTab {
  double c[3][4][4];
  double sp[2][4];
  double w[4];
  double d[4][4];   // D itself (operator entries of the matrix-core z-contractions)
  double szt[4][4]; // [a][b] = D[b][a] / w_a for b in {0, 3}, else 0: the SIPG spread along a line
};
constexpr CoefTab make_coef_tab() {
  CoefTab t{};
  for (int a = 0; a < 4; ++a) {
    for (int r = 0; r < 4; ++r) {
      t.c[0][a][r] = CX(a, r);
      t.c[1][a][r] = CY(a, r);
      t.c[2][a][r] = CZ(a, r);
    }
    t.sp[0][a] = GLL.D[0][a] / GLL.w[a];
    t.sp[1][a] = GLL.D[3][a] / GLL.w[a];
    t.w[a] = GLL.w[a];
    for (int b = 0; b < 4; ++b) {
      t.d[a][b] = GLL.D[a][b];
      t.szt[a][b] = (b == 0 || b == 3) ? GLL.D[b][a] / GLL.w[a] : 0.0;
    }
  }
  return t;
}
static __constant__ CoefTab kCoef = make_coef_tab();

struct KArgs {
  long long E;
  long long nblocks;    // logical workgroups of the element passes
  long long xcd_chunk;  // logical workgroups per XCD slab
  int N[3];
  // hexahedron stage pass: x-y tile of its traversal order (see tiled_coords)
  int tile[2];
  int bc[3][2];
  // the same boundary kinds, 3 bits per side at bit 3 (2k + side): read with
  // a per-lane side as a shift of a kernel argument (bc_kind), not as an
  // indexed load that the compiler would wait for at once
  unsigned bc_bits;
  double bcs[3][2][8];
  double Jinv[3];
  double lift[3];       // 1 / (w_0 J_k): face-to-node lift under GLL collocation
  double pen[3];        // c_ip (p+1)^2 / h_k
  double J[3];          // h_k / 2
  double hJ2inv[3];     // 1 / (2 J_k^2) (SIPG symmetric term)
  // stiffened-gas closure and mixture rules
  double xi1, xi2;      // 1 / (gamma_l - 1)
  double pi1, pi2;      // gamma_l Pinf_l / (gamma_l - 1)
  double gh1, gh2;      // gamma_l / (gamma_l - 1)
  double pinf1, pinf2;
  double rho01, rho02;  // rho_l^(0)
  double Gamma, eps, GammaEps;
  double mu1, mu2, sigma;
  double grav[3];
  double delta;         // regulariser of |grad psi| and |grad alpha|
  int has_grav;
  // stage combination U_out = rk_a U_n + rk_b (U_s + dt R)
  double rk_a, rk_b;
  // reference values of the monitor deviations
  double p_ref, u_ref[3];
  // time-step rule of a fused step (dt reduced inside the first stage)
  double cfl, hmin;
  long long nrate;  // number of rate records
  // quadrilaterals of degree != 3: the GLL weights and derivative matrix
  // (D[i][b] = l_b'(xi_i)), built on the host
  double gw[8];
  double gD[8][8];
};

// Boundary kind of side `side` of axis k (both may vary between lanes).
__device__ __forceinline__ int bc_kind(const KArgs& A, int k, int side) {
  return (int)((A.bc_bits >> (3 * (2 * k + side))) & 7u);
}

struct StageIO {
  const double* Us;   // stage input state
  const double* Gin;  // face ingredients of Us
  const double* Un;   // U^n (stage combination)
  double* Out;        // R or the new stage state
  double* Gout;       // face ingredients of Out (epilogue)
  double* rec;        // reduction records (epilogue)
  const double* dt;   // device time step
  // fused time step (first stage only; dt_out == NULL: dt is read from *dt):
  // every workgroup reduces the rate records rate_in (or takes *dt_fixed),
  // workgroup 0 stores dt to *dt_out and adds it to *t
  const double* rate_in;
  double* dt_out;
  double* t;
  const double* dt_fixed;
  // per-step monitors on a small grid: the last stage's full records also
  // leave their rate slots in rate_out (the next first stage's rate_in), and
  // that first stage reduces the full records mon_rec into *mon_out
  double* rate_out;
  const double* mon_rec;
  dg2p_monitors* mon_out;
};

struct Prim {
  double rho, u[3], kin, P, c, sE;  // sE = rho1 H1 - rho2 H2
};

// ---- cross-lane moves of a double -------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// quad rotation: lane a of a quad receives lane (a + R) & 3
template <int R>
__device__ __forceinline__ double qrot(double v) {
  return dpp64<((0 + R) & 3) | (((1 + R) & 3) << 2) | (((2 + R) & 3) << 4) | (((3 + R) & 3) << 6)>(v);
}
// quad broadcast of lane S of each quad
template <int S>
__device__ __forceinline__ double qbcast(double v) {
  return dpp64<S | (S << 2) | (S << 4) | (S << 6)>(v);
}
// row rotation: lane i of a 16-lane row receives lane (i - 4N) mod 16
template <int N>
__device__ __forceinline__ double rrot(double v) {
  return dpp64<0x120 + 4 * N>(v);
}

// ---- reciprocal and square roots -------------------------------------------------
// FP64 reciprocal, square root and reciprocal square root from the hardware
// estimates (v_rcp_f64, v_rsq_f64) refined by two Newton-Raphson steps
// (reciprocal) or two steps of Goldschmidt's iteration (square root, with a
// final residual correction): about half the instructions of the IEEE-exact
// sequences.  Measured against IEEE division and sqrt on 4.2 M values
// spanning 2^-300 .. 2^301: the reciprocal and the square root agree bit for
// bit, the reciprocal square root is within 2 ulp.  Zero and infinity are
// outside their domain (the refinement turns 0 * inf into NaN), except that
// sqrt_nr returns a zero argument unchanged; a non-positive or infinite
// argument only occurs for a non-physical state, which the monitors count.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// g ~ sqrt(x), h ~ 1 / (2 sqrt(x))
__device__ __forceinline__ void goldschmidt(double x, double& g, double& h) {
  const double y = __builtin_amdgcn_rsq(x);
  g = x * y;
  h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
}
__device__ __forceinline__ double sqrt_nr(double x) {
  double g, h;
  goldschmidt(x, g, h);
  const double d = fma(-g, g, x);
  return x == 0.0 ? x : fma(d, h, g);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double g, h;
  goldschmidt(x, g, h);
  return 2.0 * h;
}

// Per-lane rotated derivative coefficients for each axis; for hexahedra also
// the lane's entry of the z-contraction operator on the matrix cores (below).
template <int DIM>
struct LaneD {
  double c[DIM][4];
  double mz;
};

// ---- z-contractions of a hexahedron on the matrix cores ------------------------
// v_mfma_f64_4x4x4f64 multiplies four independent 4x4 FP64 blocks in one wave
// instruction: lane l supplies A[l & 3][l >> 4] and B[l >> 4][l & 3] of block
// (l >> 2) & 3 and receives C[l >> 4][l & 3] (measured on gfx950).  With the
// node index a_x + 4 a_y + 16 a_z of the lane, B = f is the field itself
// (block = a_y, row = a_z, column = a_x), so C = M f contracts every z-line of
// the element with the 4x4 operator M, and the result lands on its own node:
// no lane exchange.  A lane holds the entry M[a_x][a_z] of the operator.
__device__ __forceinline__ double mfma_z(double m, double f, double acc) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(m, f, acc, 0, 0, 0);
}

template <int DIM>
__device__ __forceinline__ void lane_coeffs(const KArgs& A, const int* ak, LaneD<DIM>& L) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
#pragma unroll
    for (int r = 0; r < 4; ++r) L.c[k][r] = kCoef.c[k][ak[k]][r];
  }
  // z-derivative operator (1/J_z) D: entry [a_x][a_z]
  L.mz = DIM == 3 ? kCoef.d[ak[0]][ak[DIM == 3 ? 2 : 0]] * A.Jinv[2] : 0.0;
}

// Sum over the 4 nodes of the lane's line along axis K of D[a_K][b] f_b.
template <int K, int DIM>
__device__ __forceinline__ double contract(double f, const LaneD<DIM>& L) {
  const double* c = L.c[K];
  if constexpr (K == 0) {
    double r = c[0] * f;
    r = fma(c[1], qrot<1>(f), r);
    r = fma(c[2], qrot<2>(f), r);
    return fma(c[3], qrot<3>(f), r);
  } else {
    static_assert(K == 1, "z-contractions run on the matrix cores (mfma_z)");
    double r = c[0] * f;
    r = fma(c[1], rrot<1>(f), r);
    r = fma(c[2], rrot<2>(f), r);
    return fma(c[3], rrot<3>(f), r);
  }
}

// Derivative along axis k: (1/J_k) sum_b D[a_k][b] f_b.  Must be called by
// the whole wave (uniform control flow): the z-contraction is a wave-wide
// matrix instruction.
template <int DIM>
__device__ __forceinline__ double dk(double f, int k, const LaneD<DIM>& L, const KArgs& A) {
  if (k == 0) return contract<0, DIM>(f, L) * A.Jinv[0];
  if constexpr (DIM > 1)
    if (k == 1) return contract<(DIM > 1 ? 1 : 0), DIM>(f, L) * A.Jinv[1];
  if constexpr (DIM > 2) return mfma_z(L.mz, f, 0.0);
  return 0.0;
}

// ---- mixed-precision contractions -------------------------------------------
// Inputs are the fluctuation f - f_ref about the element's value at its node 0
// (formed in FP64; D annihilates constants, so the result is the same
// derivative and a uniform field contracts to exactly zero), rounded to FP32
// (PR = 1) or to BF16 (PR = 2, coefficients rounded too), moved with 32-bit
// lane exchanges and accumulated in FP32.
template <int CTRL>
__device__ __forceinline__ float dpp32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u = (u + (((u >> 16) & 1u) + 0x7FFFu)) & 0xFFFF0000u;  // round to nearest even
  return __uint_as_float(u);
}
template <int DIM>
__device__ __forceinline__ double elem_ref(double f) {
  constexpr int NN = 1 << (2 * DIM);
  return __shfl(f, __lane_id() & ~(NN - 1));
}
template <int DIM>
struct LaneF {
  float c[DIM][4];
};
template <int DIM, int PR>
__device__ __forceinline__ void lane_coeffs_f(const int* ak, LaneF<DIM>& L) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float x = (float)kCoef.c[k][ak[k]][r];
      L.c[k][r] = PR == 2 ? bf16_round(x) : x;
    }
  }
}
template <int K, int DIM>
__device__ __forceinline__ float contract_f(float d, const LaneF<DIM>& L) {
  const float* c = L.c[K];
  if constexpr (K == 0) {
    float r = c[0] * d;
    r = fmaf(c[1], dpp32<0x39>(d), r);   // quad rotation by 1
    r = fmaf(c[2], dpp32<0x4E>(d), r);   // by 2
    return fmaf(c[3], dpp32<0x93>(d), r);  // by 3
  } else if constexpr (K == 1) {
    float r = c[0] * d;
    r = fmaf(c[1], dpp32<0x124>(d), r);  // row rotation by 4
    r = fmaf(c[2], dpp32<0x128>(d), r);  // by 8
    return fmaf(c[3], dpp32<0x12C>(d), r);  // by 12
  } else {
    float r = c[0] * d;
    r = fmaf(c[1], __shfl_xor(d, 16), r);
    r = fmaf(c[2], __shfl_xor(d, 32), r);
    return fmaf(c[3], __shfl_xor(d, 48), r);
  }
}

// Derivative along axis k in the precision PR (0: FP64, 1: FP32, 2: BF16 inputs).
template <int DIM, int PR>
struct Deriv {
  LaneD<DIM> L;
  LaneF<DIM> F;
};
template <int DIM, int PR>
__device__ __forceinline__ double dkp(double f, int k, const Deriv<DIM, PR>& Dv, const KArgs& A) {
  if constexpr (PR == 0) {
    return dk<DIM>(f, k, Dv.L, A);
  } else {
    float d = (float)(f - elem_ref<DIM>(f));
    if constexpr (PR == 2) d = bf16_round(d);
    float r;
    if (k == 0) r = contract_f<0, DIM>(d, Dv.F);
    else if (DIM > 1 && k == 1) r = contract_f<(DIM > 1 ? 1 : 0), DIM>(d, Dv.F);
    else r = contract_f<(DIM > 2 ? 2 : 0), DIM>(d, Dv.F);
    return (double)r * A.Jinv[k];
  }
}
template <int DIM, int PR>
__device__ __forceinline__ void deriv_setup(const KArgs& A, const int* ak, Deriv<DIM, PR>& Dv) {
  if constexpr (PR == 0)
    lane_coeffs<DIM>(A, ak, Dv.L);
  else
    lane_coeffs_f<DIM, PR>(ak, Dv.F);
}

// Value of f at the low (a_k = 0) / high (a_k = 3) end of the lane's line along k.
template <int K>
__device__ __forceinline__ double line_end(double f, int ak_k, bool high) {
  if constexpr (K == 0) {
    return high ? qbcast<3>(f) : qbcast<0>(f);
  } else if constexpr (K == 1) {
    const int lane = __lane_id();
    return __shfl(f, lane + ((high ? 3 : 0) - ak_k) * 4);
  } else {
    const int lane = __lane_id();
    return __shfl(f, lane + ((high ? 3 : 0) - ak_k) * 16);
  }
}

// ---- closure ---------------------------------------------------------------
// Stiffened-gas primitive recovery of one node: P = (rho e - Pi) / xi with the
// mixture xi = sum alpha_l/(gamma_l-1) and Pi = sum alpha_l gamma_l Pinf_l/(gamma_l-1);
// frozen mixture sound speed c^2 = ((1+xi) P + Pi) / (xi rho);
// rho_l H_l = gamma_l (P + Pinf_l)/(gamma_l-1).
template <int DIM>
__device__ __forceinline__ void closure(const KArgs& A, const double* q, Prim& p) {
  p.rho = q[0] + q[1];
  const double al = q[3 + DIM];
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
  // one division: 1/rho = xi inv and 1/xi = rho inv with inv = 1/(xi rho)
  const double inv = rcp_nr(xi * p.rho);
  const double ri = xi * inv;
  double k2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    p.u[j] = q[2 + j] * ri;
    k2 = fma(p.u[j], p.u[j], k2);
  }
  p.kin = 0.5 * k2;
  const double rhoe = q[2 + DIM] - p.rho * p.kin;
  p.P = (rhoe - pi) * (p.rho * inv);
  p.c = sqrt_nr(((1.0 + xi) * p.P + pi) * inv);
  p.sE = A.gh1 * (p.P + A.pinf1) - A.gh2 * (p.P + A.pinf2);
}

// Scalar s_q of the interface-capturing flux s_q a_1 for the conservative
// equations q = (q1, q2, rho u_j, rho E): R_1 = rho1_0 a_1, R_2 = -rho2_0 a_1,
// f (x) u with f = (rho1_0 - rho2_0) a_1, f k + (rho1 H1 - rho2 H2) a_1.
template <int DIM>
__device__ __forceinline__ double s_coef(const KArgs& A, const Prim& p, int q) {
  const double dr = A.rho01 - A.rho02;
  if (q == 0) return A.rho01;
  if (q == 1) return -A.rho02;
  if (q < 2 + DIM) return dr * p.u[q - 2];
  return dr * p.kin + p.sE;
}

// Convective flux of conservative equation q along axis k.
template <int DIM>
__device__ __forceinline__ double conv_flux(const double* q, const Prim& p, int qi, int k) {
  if (qi < 2) return q[qi] * p.u[k];
  if (qi < 2 + DIM) return q[qi] * p.u[k] + ((qi - 2) == k ? p.P : 0.0);
  return (q[2 + DIM] + p.P) * p.u[k];
}

// Index of a node inside the face layer normal to axis k (axis k removed).
__device__ __forceinline__ int face_index(int node, int k) {
  const int lowmask = (1 << (2 * k)) - 1;
  return (node & lowmask) | ((node >> (2 * k + 2)) << (2 * k));
}

// Element-local gradient quantities of a node.
template <int DIM, bool VISC>
struct Grad {
  double gA[DIM], nh[DIM], a[DIM];
  double upsi;  // u . grad psi
  double S[VISC ? DIM : 1][VISC ? DIM : 1];  // grad u + grad u^T - 2/3 div u I
  double mu;
};

template <int DIM, bool VISC, int PR>
__device__ __forceinline__ void gradients(const KArgs& A, const double* q, const Prim& p,
                                          const Deriv<DIM, PR>& L, Grad<DIM, VISC>& g) {
  const double al = q[3 + DIM];
  const double ps = q[4 + DIM];
  double gP[DIM];
  double g2 = 0.0;
  g.upsi = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    g.gA[k] = dkp<DIM, PR>(al, k, L, A);
    gP[k] = dkp<DIM, PR>(ps, k, L, A);
    g2 = fma(gP[k], gP[k], g2);
    g.upsi = fma(p.u[k], gP[k], g.upsi);
  }
  const double inv = rsqrt_nr(g2 + A.delta * A.delta);
  const double aa = al * (1.0 - al);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    g.nh[k] = gP[k] * inv;
    g.a[k] = A.Gamma * (A.eps * g.gA[k] - aa * g.nh[k]);
  }
  if constexpr (VISC) {
    double gU[DIM][DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k) gU[j][k] = dkp<DIM, PR>(p.u[j], k, L, A);
    double div = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) div += gU[j][j];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k)
        g.S[j][k] = gU[j][k] + gU[k][j] - (j == k ? (2.0 / 3.0) * div : 0.0);
    g.mu = A.mu1 * al + A.mu2 * (1.0 - al);
  } else {
    g.mu = 0.0;
  }
}

// ---- reduction helpers -----------------------------------------------------------
// Maximum and minimum that propagate NaN (fmax / fmin drop it): a node whose
// closure fails (e.g. a negative squared sound speed) turns the reduced rate,
// hence dt, and the reduced monitors into NaN, as the oracle's reductions do,
// instead of being skipped.  Exact and order-independent, like fmax.
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }
__device__ __forceinline__ double nan_min(double a, double b) { return (a < b || a != a) ? a : b; }

// ---- lane exchanges of the wave reductions, all on the vector ALU ------------
// (a few cycles of latency each, where __shfl_xor is an LDS-routed permute).
// gfx950's v_permlane32_swap(x, y) swaps the upper half-wave of x with the
// lower half-wave of y: its first result holds x[l] in lanes 0-31 and
// y[l - 32] in lanes 32-63, its second x[l + 32] in lanes 0-31 and y[l] in
// lanes 32-63; v_permlane16_swap does the same between the odd 16-lane rows
// of x and the even rows of y (first: x[l] in even rows, y[l - 16] in odd
// rows; second: x[l + 16] in even rows, y[l] in odd rows).  So with x = the
// half a lower lane keeps and y = the half an upper lane keeps, first +
// second is, in every lane, its own half combined with the partner's same
// half: one step of a reduce-scatter over lane mask 32 (16) without a select.
__device__ __forceinline__ unsigned lo32(double v) { return (unsigned)(__double_as_longlong(v) & 0xffffffffull); }
__device__ __forceinline__ unsigned hi32(double v) { return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int M>
__device__ __forceinline__ void swap_halves(double x, double y, double& a, double& b) {
  static_assert(M == 16 || M == 32, "row-pair or half-wave swap");
  if constexpr (M == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(y), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(y), false, false);
    a = mk64(l[0], h[0]);
    b = mk64(l[1], h[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(y), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(y), false, false);
    a = mk64(l[0], h[0]);
    b = mk64(l[1], h[1]);
  }
}
// value of lane l ^ M for M < 16 (inside a 16-lane row).  The DPP row
// rotation by R gives lane l the value of lane (l - R) mod 16 of its row, so
// the rotation by 8 is xor 8, and xor 4 is the rotation by 12 (l + 4, lanes
// with bit 2 clear) or by 4 (l - 4, bit 2 set); xor 2 and xor 1 are quad
// permutations
template <int M>
__device__ __forceinline__ double xor_lane(double v) {
  if constexpr (M == 8) {
    return rrot<2>(v);
  } else if constexpr (M == 4) {
    const double back = rrot<1>(v), fwd = rrot<3>(v);
    return (__lane_id() & 4) ? back : fwd;
  } else if constexpr (M == 2) {
    return dpp64<0x4E>(v);
  } else {
    static_assert(M == 1, "lane mask 1, 2, 4 or 8");
    return dpp64<0xB1>(v);
  }
}
// OP over the whole wave, result in every lane (0 sum, 1 max, 2 min; the
// maximum and minimum keep NaN)
template <int OP>
__device__ __forceinline__ double wave_op2(double a, double b) {
  return OP == 0 ? a + b : (OP == 1 ? nan_max(a, b) : nan_min(a, b));
}
template <int OP>
__device__ __forceinline__ double wave_all(double v) {
  double a, b;
  swap_halves<32>(v, v, a, b);
  v = wave_op2<OP>(a, b);
  swap_halves<16>(v, v, a, b);
  v = wave_op2<OP>(a, b);
  v = wave_op2<OP>(v, xor_lane<8>(v));
  v = wave_op2<OP>(v, xor_lane<4>(v));
  v = wave_op2<OP>(v, xor_lane<2>(v));
  return wave_op2<OP>(v, xor_lane<1>(v));
}
__device__ __forceinline__ double wave_max(double v) { return wave_all<1>(v); }
__device__ __forceinline__ double wave_min(double v) { return wave_all<2>(v); }
__device__ __forceinline__ double wave_sum(double v) { return wave_all<0>(v); }

// Rate record of a workgroup (2 doubles: largest wave speed and largest
// kinematic viscosity): wave max, then the workgroup's 4 waves.
constexpr int RATE = 2;
template <int WT = BLOCK>
__device__ __forceinline__ void block_rate_record(double w, double nu, double* rec, long long blk) {
  __shared__ double sh[2][WT / 64];
  w = wave_max(w);
  nu = wave_max(nu);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = w;
    sh[1][threadIdx.x >> 6] = nu;
  }
  __syncthreads();
  if (threadIdx.x < RATE) {
    const int s = threadIdx.x;  // R_WAVE, R_NU
    double x = sh[s][0];
#pragma unroll
    for (int i = 1; i < WT / 64; ++i) x = nan_max(x, sh[s][i]);
    rec[blk * RATE + s] = x;
  }
}

// Time-step rule from the reduced maxima: rate = (max wave + (p+1)^2 d
// nu_max / h_min) / h_min with nu_max = max(Gamma eps, max mu/rho);
// pdim = (p+1)^2 d.
__device__ __forceinline__ double rate_of(double wmax, double numax, double GammaEps, double pdim, double hmin) {
  const double nu = nan_max(GammaEps, numax);
  return (wmax + pdim * nu / hmin) / hmin;
}

// Fused time step of a small grid: every workgroup reduces all rate records
// (max is exact, so every workgroup obtains the same value as the separate
// reduction kernels). First half, at kernel entry so that the record loads
// overlap those of the stage input: each thread's maximum over its share of
// the records (independent loads), then its wave's maximum, parked in LDS.
constexpr int FUSED_RATE_PER_THREAD = 4;
constexpr long long FUSED_RATE_MAX = FUSED_RATE_PER_THREAD * BLOCK;  // records a four-wave workgroup reduces
template <int WT>
__device__ __forceinline__ void fused_dt_load(const KArgs& A, const double* __restrict__ rate,
                                              double (*sh)[WT / 64]) {
  // A.nrate <= FUSED_RATE_MAX: straight-line loads (clamped to record 0,
  // their values discarded), no loop whose latch would wait for every load
  double vw[FUSED_RATE_PER_THREAD], vn[FUSED_RATE_PER_THREAD];
#pragma unroll
  for (int u = 0; u < FUSED_RATE_PER_THREAD; ++u) {
    const long long r = threadIdx.x + u * WT;
    const long long rr = r < A.nrate ? r : 0;
    vw[u] = rate[rr * RATE + R_WAVE];
    vn[u] = rate[rr * RATE + R_NU];
  }
  double w = 0.0, nu = 0.0;
#pragma unroll
  for (int u = 0; u < FUSED_RATE_PER_THREAD; ++u) {
    const bool ok = threadIdx.x + u * WT < A.nrate;
    w = nan_max(w, ok ? vw[u] : 0.0);
    nu = nan_max(nu, ok ? vn[u] : 0.0);
  }
  w = wave_max(w);
  nu = wave_max(nu);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = w;
    sh[1][threadIdx.x >> 6] = nu;
  }
}

// Second half, at the stage combine (the first point that needs dt, so that
// the workgroup barrier does not hold the waves back at entry): the maxima
// over the workgroup's waves, and the rate from them (dt = cfl / rate).
// pdim = (p+1)^2 d of the time-step rule.
template <int WT>
__device__ __forceinline__ double fused_rate_finish(const KArgs& A, double (*sh)[WT / 64], double pdim) {
  __syncthreads();
  double w = sh[0][0];
  double nu = sh[1][0];
#pragma unroll
  for (int i = 1; i < WT / 64; ++i) {
    w = nan_max(w, sh[0][i]);
    nu = nan_max(nu, sh[1][i]);
  }
  return rate_of(w, nu, A.GammaEps, pdim, A.hmin);
}

// Per-node record contributions of a state (time-step rate and monitors), W
// the node's quadrature weight.
template <int DIM, bool VISC>
__device__ __forceinline__ void node_record_w(const KArgs& A, const double* q, const Prim& p, double W,
                                              bool valid, double* v) {
  constexpr int NF = DIM + 5;
  double w = DIM * p.c;
#pragma unroll
  for (int j = 0; j < DIM; ++j) w += fabs(p.u[j]);
  const double al = q[3 + DIM];
  double nu = 0.0;
  if constexpr (VISC) nu = (A.mu1 * al + A.mu2 * (1.0 - al)) * rcp_nr(p.rho);
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
  const bool bad = !(p.rho > 0.0) || !(xi * p.rho > 0.0) || !((1.0 + xi) * p.P + pi > 0.0) ||
                   !isfinite(p.P) || !isfinite(p.c);
  double du = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) du = nan_max(du, fabs(p.u[j] - A.u_ref[j]));
  v[R_WAVE] = valid ? w : 0.0;
  v[R_NU] = valid ? nu : 0.0;
  v[R_AMIN] = valid ? al : INFINITY;
  v[R_AMAX] = valid ? al : -INFINITY;
  v[R_BAD] = (valid && bad) ? 1.0 : 0.0;
  v[R_DEVP] = valid ? fabs(p.P - A.p_ref) : 0.0;
  v[R_DEVU] = valid ? du : 0.0;
#pragma unroll
  for (int f = 0; f < 8; ++f) v[R_INT + f] = (valid && f < NF) ? W * q[f] : 0.0;
}

// The same for a node of the p = 3 lane layout (node = sum_k a_k 4^k).
template <int DIM, bool VISC>
__device__ __forceinline__ void node_record(const KArgs& A, const double* q, const Prim& p, int node,
                                            bool valid, double* v) {
  double W = 1.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int a = (node >> (2 * k)) & 3;
    W *= ((a == 0 || a == 3) ? GLL.w[0] : GLL.w[1]) * A.J[k];
  }
  node_record_w<DIM, VISC>(A, q, p, W, valid, v);
}

__device__ __forceinline__ double rec_combine(int slot, double a, double b) {
  if (slot == R_AMIN) return nan_min(a, b);
  if (slot == R_WAVE || slot == R_NU || slot == R_AMAX || slot == R_DEVP || slot == R_DEVU) return nan_max(a, b);
  return a + b;
}
__device__ __forceinline__ double rec_identity(int slot) {
  return slot == R_AMIN ? INFINITY : (slot == R_AMAX ? -INFINITY : 0.0);
}
__device__ __forceinline__ double rec_wave(int slot, double v) {
  if (slot == R_AMIN) return wave_min(v);
  if (slot == R_WAVE || slot == R_NU || slot == R_AMAX || slot == R_DEVP || slot == R_DEVU) return wave_max(v);
  return wave_sum(v);
}

// Reduce-scatter of NS per-lane values over the wave (NS a power of two,
// 8 or 16): butterfly over lane masks 32, 16, ... that halves the number of
// slots a lane carries at every step, then a plain butterfly over the
// remaining mask bits.  Afterwards every lane l holds the wave-wide result of
// slot l >> (6 - log2 NS).  OP: 0 = sum, 1 = max.
// one step over lane mask M: lanes with that bit clear keep the low half of
// v (v[0..HALF)), the others the high half, each combined with its partner's
// same half (lane exchanges on the vector ALU, above)
template <int HALF, int M, int OP>
__device__ __forceinline__ void rs_step(double* v) {
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const double lo = v[i], hi = v[HALF + i];
    if constexpr (M >= 16) {
      double a, b;
      swap_halves<M>(lo, hi, a, b);
      v[i] = wave_op2<OP>(a, b);
    } else {
      const bool upper = (__lane_id() & M) != 0;
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      v[i] = wave_op2<OP>(keep, xor_lane<M>(send));
    }
  }
}
template <int OP, int M>
__device__ __forceinline__ double bfly(double x) {
  return wave_op2<OP>(x, xor_lane<M>(x));
}
template <int NS, int OP>
__device__ __forceinline__ double wave_reduce_scatter(double* v) {
  if constexpr (NS == 16) {
    rs_step<8, 32, OP>(v);
    rs_step<4, 16, OP>(v);
    rs_step<2, 8, OP>(v);
    rs_step<1, 4, OP>(v);
    return bfly<OP, 1>(bfly<OP, 2>(v[0]));
  } else {
    static_assert(NS == 8, "reduce-scatter of 8 or 16 slots");
    rs_step<4, 32, OP>(v);
    rs_step<2, 16, OP>(v);
    rs_step<1, 8, OP>(v);
    return bfly<OP, 1>(bfly<OP, 2>(bfly<OP, 4>(v[0])));
  }
}

// Workgroup reduction of per-lane records into rec[blk * REC + slot] (fixed
// order); if rate != NULL its rate slots also into rate[blk * RATE + slot].
template <int WT = BLOCK>
__device__ __forceinline__ void block_record(double* v, double* rec, long long blk, double* rate = nullptr) {
  __shared__ double sh[REC][WT / 64];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  // max group: wave, nu, -min alpha, max alpha, dev p, dev u (padded to 8)
  double mx[8] = {v[R_WAVE], v[R_NU], -v[R_AMIN], v[R_AMAX], v[R_DEVP], v[R_DEVU], -INFINITY, -INFINITY};
  // sum group: non-physical count and the 8 integral slots (padded to 16)
  double sm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) sm[i] = 0.0;
  sm[0] = v[R_BAD];
#pragma unroll
  for (int f = 0; f < 8; ++f) sm[1 + f] = v[R_INT + f];
  const double xm = wave_reduce_scatter<8, 1>(mx);
  const double xs = wave_reduce_scatter<16, 0>(sm);
  if ((lane & 7) == 0) {
    // slots 0..5 of the max group: R_WAVE, R_NU, R_AMIN, R_AMAX, R_DEVP, R_DEVU
    const int slot = lane >> 3;
    const int dst = slot < 4 ? slot : slot + (R_DEVP - 4);
    if (slot < 6) sh[dst][w] = slot == 2 ? -xm : xm;
  }
  if ((lane & 3) == 0) {
    const int slot = lane >> 2;
    if (slot == 0) sh[R_BAD][w] = xs;
    else if (slot <= 8) sh[R_INT + slot - 1][w] = xs;
  }
  __syncthreads();
  if (threadIdx.x < REC) {
    const int s = threadIdx.x;
    double x = sh[s][0];
#pragma unroll
    for (int i = 1; i < WT / 64; ++i) x = rec_combine(s, x, sh[s][i]);
    rec[blk * REC + s] = x;
    if (rate && s < RATE) rate[blk * RATE + s] = x;  // R_WAVE, R_NU
  }
}

// Grid coordinates of element e (x fastest). Element counts are below 2^31
// (checked when the mesh is created), so 32-bit unsigned division suffices.
template <int DIM>
__device__ __forceinline__ void elem_coords(const KArgs& A, long long e, long long* ec) {
  unsigned r = (unsigned)e;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const unsigned n = (unsigned)A.N[k];
    ec[k] = r % n;
    r /= n;
  }
}

// Side of the x-y tiles of the hexahedron stage pass's traversal order.
#ifndef DG2P_TILE_3D
#define DG2P_TILE_3D 16
#endif

// Logical workgroup of this physical workgroup (XCD-aware order); -1 if padding.
__device__ __forceinline__ long long logical_block(const KArgs& A) {
  const long long i = blockIdx.x;
  const long long lb = (i & 7) * A.xcd_chunk + (i >> 3);
  return lb < A.nblocks ? lb : -1;
}

// Element (multi-index ec) of logical workgroup lb of the hexahedron stage
// pass (one element each).  The x-y plane is cut into tiles of A.tile[0] x
// A.tile[1] elements (cut short at the high edges), taken row of tiles by
// row of tiles, each tile through all its z-layers before the next, a layer
// in x-fastest order.  An element's z-neighbours then come one tile-layer
// apart in the order instead of one whole x-y layer (9216 elements on a 96^3
// box), close enough for the cache to still hold the face traces they read
// of each other; with the tile the whole x-y layer, the order is the
// storage order.
__device__ __forceinline__ void tiled_coords(const KArgs& A, unsigned lb, long long* ec) {
  const unsigned n0 = (unsigned)A.N[0], n1 = (unsigned)A.N[1], n2 = (unsigned)A.N[2];
  const unsigned tx = (unsigned)A.tile[0], ty = (unsigned)A.tile[1];
  const unsigned rowsz = n0 * ty * n2;  // a full row of tiles (<= E < 2^31)
  const unsigned r = lb / rowsz;
  unsigned rem = lb - r * rowsz;
  const unsigned y0 = r * ty;
  const unsigned h = min(ty, n1 - y0);
  const unsigned colsz = tx * h * n2;  // a full tile of this row, all layers
  const unsigned c = rem / colsz;
  rem -= c * colsz;
  const unsigned x0 = c * tx;
  const unsigned w = min(tx, n0 - x0);
  const unsigned lay = w * h;
  const unsigned z = rem / lay;
  rem -= z * lay;
  const unsigned yy = rem / w;
  ec[0] = x0 + (rem - yy * w);
  ec[1] = y0 + yy;
  ec[2] = z;
}

// Launch arguments of the stage pass: the traversal tile of hexahedra.
template <int DIM>
inline KArgs stage_args(const KArgs& A) {
  KArgs B = A;
  B.tile[0] = (DIM == 3 && DG2P_TILE_3D < A.N[0]) ? DG2P_TILE_3D : A.N[0];
  B.tile[1] = (DIM == 3 && DG2P_TILE_3D < A.N[1]) ? DG2P_TILE_3D : A.N[1];
  return B;
}

// Stores of a pass's outputs (the next state, its face ingredients).  On
// hexahedra they are streamed past the caches: nothing reads them again in
// the same pass, while the pass's own input is re-read by the neighbours' face
// loads, which the outputs would otherwise evict (96^3: -1.2 % per stage).
template <int DIM>
__device__ __forceinline__ void store_out(double* p, double v) {
  if constexpr (DIM == 3) __builtin_nontemporal_store(v, p);
  else *p = v;
}
typedef double dbl2 __attribute__((ext_vector_type(2)));
template <int DIM>
__device__ __forceinline__ void store_out2(double* p, dbl2 v) {
  if constexpr (DIM == 3) __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(p));
  else *reinterpret_cast<dbl2*>(p) = v;
}

// Layout of the face-ingredient buffer G.  Face slot s = 2k + side of an
// element holds, at each of its NFN face nodes, C components: a.e_k, then
// (viscous) the traction mu S[j][k], j < d.  They are stored in pairs (W = 2;
// one value when C = 1), so that a lane moves its node's ingredients with one
// 16-byte access per pair, and element by element:
// G[((e 2d + s) P + pr) NFN W + fn W + i] holds component pr W + i.  An
// element's ingredients are one contiguous block (3 KB for a viscous
// hexahedron), so a pass writes G as one stream instead of one per face slot
// and component.
template <int DIM, bool VISC>
struct GLay {
  static constexpr int C = VISC ? 1 + DIM : 1;
  static constexpr int W = C == 1 ? 1 : 2;
  static constexpr int P = (C + W - 1) / W;
  static constexpr int NFN = (1 << (2 * DIM)) / 4;
  __device__ static long long at(long long E, int slot, int pr, long long e, int fn) {
    (void)E;
    return ((e * (2 * DIM) + slot) * P + pr) * (NFN * W) + (long long)fn * W;
  }
};
// The ingredients of face slot `slot`, node fn of element e: v[0] = a.e_k,
// v[1 + j] = the traction components.  NT: a non-temporal load (a slot is
// read by one element only, the neighbour across its face, so on hexahedra
// it need not displace the states the neighbours still read from the cache).
template <int DIM, bool VISC, bool NT = false>
__device__ __forceinline__ void g_read(const KArgs& A, const double* __restrict__ G, int slot, long long e, int fn,
                                       double* v) {
  using L = GLay<DIM, VISC>;
  if constexpr (L::W == 2) {
#pragma unroll
    for (int pr = 0; pr < L::P; ++pr) {
      const dbl2* p = reinterpret_cast<const dbl2*>(G + L::at(A.E, slot, pr, e, fn));
      dbl2 x;
      if constexpr (NT) x = __builtin_nontemporal_load(p);
      else x = *p;
      v[2 * pr] = x.x;
      v[2 * pr + 1] = x.y;
    }
  } else {
    if constexpr (NT) v[0] = __builtin_nontemporal_load(G + L::at(A.E, slot, 0, e, fn));
    else v[0] = G[L::at(A.E, slot, 0, e, fn)];
  }
}

// ---- epilogue: face ingredients and records of a state held per lane ----------------
template <int DIM, bool VISC, bool WRITE_G, int REC_MODE, int PR>
__device__ __forceinline__ void emit(const KArgs& A, const double* q, long long e, bool valid, int node,
                                     const int* ak, const Deriv<DIM, PR>& L, double* G, double* rec,
                                     long long blk, double* rate = nullptr) {
  Prim p;
  closure<DIM>(A, q, p);
  if constexpr (WRITE_G) {
    Grad<DIM, VISC> g;
    gradients<DIM, VISC, PR>(A, q, p, L, g);
    if (valid) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if (ak[k] != 0 && ak[k] != 3) continue;
        const int side = ak[k] == 3;
        const int fn = face_index(node, k);
        using GL = GLay<DIM, VISC>;
        if constexpr (GL::W == 2) {
          double v[2 * GL::P];
          v[0] = g.a[k];
#pragma unroll
          for (int j = 0; j < DIM; ++j) v[1 + j] = g.mu * g.S[j][k];
#pragma unroll
          for (int i = 1 + DIM; i < 2 * GL::P; ++i) v[i] = 0.0;
#pragma unroll
          for (int pr = 0; pr < GL::P; ++pr)
            store_out2<DIM>(&G[GL::at(A.E, 2 * k + side, pr, e, fn)], dbl2{v[2 * pr], v[2 * pr + 1]});
        } else {
          store_out<DIM>(&G[GL::at(A.E, 2 * k + side, 0, e, fn)], g.a[k]);
        }
      }
    }
  }
  if constexpr (REC_MODE == 2) {
    double v[REC];
    node_record<DIM, VISC>(A, q, p, node, valid, v);
    block_record<ewg<DIM>()>(v, rec, blk, rate);
  } else if constexpr (REC_MODE == 1) {
    // time-step rate only: largest wave speed and kinematic viscosity
    double w = DIM * p.c;
#pragma unroll
    for (int j = 0; j < DIM; ++j) w += fabs(p.u[j]);
    double nu = 0.0;
    if constexpr (VISC) {
      const double al = q[3 + DIM];
      nu = (A.mu1 * al + A.mu2 * (1.0 - al)) * rcp_nr(p.rho);
    }
    block_rate_record<ewg<DIM>()>(valid ? w : 0.0, valid ? nu : 0.0, rec, blk);
  }
}

// ---------------------------------------------------------------------------
// Ingredient pass: G and records of a state (first stage of a step, residual).
template <int DIM, bool VISC, int PR>
__global__ __launch_bounds__(ewg<DIM>()) void k_ingredients(KArgs A, const double* __restrict__ U,
                                                       double* __restrict__ G, double* __restrict__ rec) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  const long long blk = logical_block(A);
  if (blk < 0) return;
  const int lane = threadIdx.x & 63;
  const long long e0 = (blk * (ewg<DIM>() / 64) + (threadIdx.x >> 6)) * EPW + lane / NN;
  const bool valid = e0 < A.E;
  const long long e = valid ? e0 : A.E - 1;
  const int node = lane % NN;
  int ak[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) ak[k] = (node >> (2 * k)) & 3;
  Deriv<DIM, PR> L;
  deriv_setup<DIM, PR>(A, ak, L);
  double q[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) q[f] = U[(f * A.E + e) * NN + node];
  emit<DIM, VISC, true, 1, PR>(A, q, e, valid, node, ak, L, G, rec, blk);
}

// ---- face fluxes ------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ double pick(const double* v, int k) {
  if constexpr (DIM == 1) {
    return v[0];
  } else if constexpr (DIM == 2) {
    return k ? v[1] : v[0];
  } else {
    return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
  }
}

// The same for a kernel-argument array (uniform values) with an axis that
// may vary between lanes: both candidates are pinned in scalar registers
// first, so that the selection stays a per-lane select of scalars (the
// compiler would otherwise turn it into a per-lane load from the argument
// segment, waited for at once).
template <int DIM>
__device__ __forceinline__ double pick_arg(const double* v, int k) {
  if constexpr (DIM == 1) {
    return v[0];
  } else {
    double a = v[0], b = v[1];
    asm volatile("" : "+s"(a), "+s"(b));
    if constexpr (DIM == 2) {
      return k ? b : a;
    } else {
      double c = v[2];
      asm volatile("" : "+s"(c));
      return k == 0 ? a : (k == 1 ? b : c);
    }
  }
}

// Convective flux of conservative equation qi along axis kd (velocity
// component uk = u_kd).
template <int DIM>
__device__ __forceinline__ double conv_flux_k(const double* q, const Prim& p, int qi, int kd, double uk) {
  if (qi < 2) return q[qi] * uk;
  if (qi < 2 + DIM) return q[qi] * uk + ((qi - 2) == kd ? p.P : 0.0);
  return (q[2 + DIM] + p.P) * uk;
}

// Neighbour trace across a face: the state at node nodee of element en and
// the face ingredients it published for face node fn of its side facing back
// (a.e_kd, and the viscous traction when VISC).
template <int DIM, bool VISC>
__device__ __forceinline__ void face_load(const KArgs& A, const double* __restrict__ Us,
                                          const double* __restrict__ Gin, int kd, int side, long long en, int nodee,
                                          int fn, double* qn, double& an, double* tn) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int NF = DIM + 5;
#pragma unroll
  for (int f = 0; f < NF; ++f) qn[f] = Us[(f * A.E + en) * NN + nodee];
  double v[2 * GLay<DIM, VISC>::P];
  g_read<DIM, VISC, DIM == 3>(A, Gin, 2 * kd + 1 - side, en, fn, v);
  an = v[0];
#pragma unroll
  for (int j = 0; j < DIM; ++j) tn[j] = VISC ? v[1 + j] : 0.0;
}

// Contributions of one face node of an element to that node: Rc[f] (lift
// factor included) for every field, and the SIPG symmetric-term values symv
// (conservative equations, then alpha) to be spread along the normal line.
// Face normal axis kd, side 0 (low) / 1 (high).  The element's own trace:
// q, p, a.e_kd (a_k), the viscous traction mu S[j][kd] (mu, Sk) and, for
// Dirichlet ghosts, d_kd alpha and n_kd (gA_k, nh_k).  The neighbour's trace
// is qn with its ingredients an (a.e_kd) and tn (traction), as loaded by
// face_load, or is built as the boundary ghost when bnd.
template <int DIM, bool VISC, int BCK>
__device__ __forceinline__ void face_flux(const KArgs& A, int kd, int side, bool bnd, const double* qn, double an,
                                          const double* tn, const double* q, const Prim& pr, double a_k, double mu,
                                          const double* Sk, double gA_k, double nh_k, double* Rc, double* symv) {
  constexpr int NF = DIM + 5;
  constexpr int NC = DIM + 3;
  const double sm = side ? 1.0 : -1.0;
  double qe[NF];
  double aek;
  double tek[DIM];
  if (BCK == 0 || !bnd) {
#pragma unroll
    for (int f = 0; f < NF; ++f) qe[f] = qn[f];
    aek = an;
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) tek[j] = tn[j];
    }
  } else {
    const int kind = bc_kind(A, kd, side);
#pragma unroll
    for (int f = 0; f < NF; ++f) qe[f] = q[f];
    aek = a_k;
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) tek[j] = mu * Sk[j];
    }
    if (kind == DG2P_BC_SLIP_WALL || kind == DG2P_BC_NO_SLIP) {
      // mirror image; the slip wall flips the normal momentum and mirrors the
      // shear (tangential traction negated), the no-slip wall flips the whole
      // momentum and keeps the shear
      const bool slip = kind == DG2P_BC_SLIP_WALL;
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        if (!slip || j == kd) qe[2 + j] = -q[2 + j];
      aek = -a_k;
      if constexpr (VISC) {
#pragma unroll
        for (int j = 0; j < DIM; ++j)
          if (slip && j != kd) tek[j] = -tek[j];
      }
    }
    if constexpr (BCK == 2) {
      if (kind == DG2P_BC_RIEMANN) {
        // far field at rest with pressure P_b: invariants u.n +- 2 xi c of the
        // mixture stiffened gas at the interior composition and density
        const double al = q[3 + DIM];
        const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
        const double pim = al * A.pi1 + (1.0 - al) * A.pi2;
        const double Pb = A.bcs[kd][side][0];
        const double un = sm * pick<DIM>(pr.u, kd);
        const double cfar = sqrt(((1.0 + xi) * Pb + pim) / (xi * pr.rho));
        const double jout = un + 2.0 * xi * pr.c;
        const double jin = -2.0 * xi * cfar;
        const double unb = 0.5 * (jout + jin);
        const double cb = (jout - jin) / (4.0 * xi);
        const double Pg = (xi * pr.rho * cb * cb - pim) / (1.0 + xi);
        double k2 = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          const double ug = pr.u[j] + (j == kd ? sm * (unb - un) : 0.0);
          qe[2 + j] = pr.rho * ug;
          k2 += ug * ug;
        }
        qe[2 + DIM] = xi * Pg + pim + 0.5 * pr.rho * k2;
      }
      if (kind == DG2P_BC_DIRICHLET) {
#pragma unroll
        for (int f = 0; f < 4 + DIM; ++f) qe[f] = A.bcs[kd][side][f];
        const double ag = qe[3 + DIM];
        aek = A.Gamma * (A.eps * gA_k - (ag * (1.0 - ag)) * nh_k);
        if constexpr (VISC) {
          const double mug = A.mu1 * ag + A.mu2 * (1.0 - ag);
#pragma unroll
          for (int j = 0; j < DIM; ++j) tek[j] = mug * Sk[j];
        }
      }
    }
  }
  Prim pe;
  closure<DIM>(A, qe, pe);
  const double uIk = pick<DIM>(pr.u, kd), uEk = pick<DIM>(pe.u, kd);
  const double umI = sm * uIk, umE = sm * uEk;
  const double lam = fmax(fabs(umI) + pr.c, fabs(umE) + pe.c);
  const double amI = sm * a_k, amE = sm * aek;
  const double alI = q[3 + DIM], alE = qe[3 + DIM];
  const double jump = alI - alE;
  const double penk = pick_arg<DIM>(A.pen, kd);
  const double ahat = 0.5 * (amI + amE) - penk * A.GammaEps * jump;
  const double Lf = pick_arg<DIM>(A.lift, kd);
  double etav = 0.0;
  if constexpr (VISC) {
    const double mue = A.mu1 * alE + A.mu2 * (1.0 - alE);
    etav = penk * (0.5 * (mu + mue));
  }
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) {
    const double FmI = sm * conv_flux_k<DIM>(q, pr, qi, kd, uIk);
    const double FmE = sm * conv_flux_k<DIM>(qe, pe, qi, kd, uEk);
    const double Fhat = 0.5 * (FmI + FmE) - 0.5 * lam * (qe[qi] - q[qi]);
    const double sI = s_coef<DIM>(A, pr, qi), sE = s_coef<DIM>(A, pe, qi);
    const double sbar = 0.5 * (sI + sE);
    double t = (FmI - Fhat) + (sbar * ahat - sI * amI);
    if constexpr (VISC) {
      if (qi >= 2) {
        double VmI, VmE, pen;
        if (qi < 2 + DIM) {
          const int j = qi - 2;
          VmI = sm * (mu * Sk[j]);
          VmE = sm * tek[j];
          pen = etav * (pr.u[j] - pe.u[j]);
        } else {
          double tuI = 0.0, tuE = 0.0, du = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            tuI += (mu * Sk[j]) * pr.u[j];
            tuE += tek[j] * pe.u[j];
            du += (pr.u[j] - pe.u[j]) * (0.5 * (pr.u[j] + pe.u[j]));
          }
          VmI = sm * tuI;
          VmE = sm * tuE;
          pen = etav * du;
        }
        const double Vhat = 0.5 * (VmI + VmE) - pen;
        t += Vhat - VmI;
      }
    }
    Rc[qi] = Lf * t;
    symv[qi] = sm * sbar * A.GammaEps * jump;
  }
  const double KA = 0.5 * (lam - umI) * (alE - alI);
  Rc[3 + DIM] = Lf * (KA + (ahat - amI));
  symv[NC] = sm * A.GammaEps * jump;
  Rc[4 + DIM] = Lf * (0.5 * (lam - umI) * (qe[4 + DIM] - q[4 + DIM]));
}

// One of four compile-time values by a lane's node position a (selects, no
// table load: a load here would be waited for at once, and the in-order
// memory counters would make that wait drain every load in flight).
__device__ __forceinline__ double pick4(int a, double v0, double v1, double v2, double v3) {
  double v = v0;
  v = a == 1 ? v1 : v;
  v = a == 2 ? v2 : v;
  return a == 3 ? v3 : v;
}
// SIPG spread weights D[end][a] / w_a of the line's low (end 0) and high
// (end 3) face
__device__ __forceinline__ double spread_lo(int a) {
  return pick4(a, GLL.D[0][0] / GLL.w[0], GLL.D[0][1] / GLL.w[1], GLL.D[0][2] / GLL.w[2], GLL.D[0][3] / GLL.w[3]);
}
__device__ __forceinline__ double spread_hi(int a) {
  return pick4(a, GLL.D[3][0] / GLL.w[0], GLL.D[3][1] / GLL.w[1], GLL.D[3][2] / GLL.w[2], GLL.D[3][3] / GLL.w[3]);
}

// SIPG symmetric term: the values symv of the face nodes at the two ends of
// each line along K, weighted with D[end][a] / (2 w_a J_K^2) (end = 0 for the
// low face, 3 for the high face), added to every node a of the line.
template <int K, int DIM>
__device__ __forceinline__ void spread_sym(const KArgs& A, int akk, const double* symv, double* R) {
  constexpr int NC = DIM + 3;
  if constexpr (K == 2) {
    // hexahedron z-lines on the matrix cores: R += S symv with
    // S[a][b] = D[b][a] / (2 w_a J_z^2) for the line ends b in {0, 3}
    // (akk is a_z; the lane's operator entry is S[a_x][a_z])
    const int ax = __lane_id() & 3;
    const double m = (akk == 0 ? spread_lo(ax) : (akk == 3 ? spread_hi(ax) : 0.0)) * A.hJ2inv[2];
#pragma unroll
    for (int i = 0; i <= NC; ++i) {
      const int f = (i < NC) ? i : 3 + DIM;
      R[f] = mfma_z(m, symv[i], R[f]);
    }
    return;
  }
  const double wlo = spread_lo(akk) * A.hJ2inv[K];
  const double whi = spread_hi(akk) * A.hJ2inv[K];
#pragma unroll
  for (int i = 0; i <= NC; ++i) {
    const double lo = line_end<K>(symv[i], akk, false);
    const double hi = line_end<K>(symv[i], akk, true);
    const int f = (i < NC) ? i : 3 + DIM;
    R[f] = fma(lo, wlo, fma(hi, whi, R[f]));
  }
}

// Per-step monitors of a small grid, in the first stage of the next step:
// logical workgroup b reduces the record slots R_AMIN + b, R_AMIN + b +
// nblocks, ... below R_INT + 8 over all A.nrate (<= FUSED_RATE_PER_THREAD WT)
// records in a fixed order (each thread its records in turn, then the wave,
// then the waves) and stores them into *mon; the rate and dt come from the
// fused time step (workgroup 0).  Called by whole workgroups after their
// stores; the loop bound is uniform.  The host fuses only grids of at least
// MON_SLOTS workgroups, so that no workgroup reduces more than one slot.
constexpr int MON_SLOTS = R_INT + 8 - R_AMIN;
template <int WT, int NF>
__device__ __forceinline__ void fused_monitor_slots(const KArgs& A, const double* __restrict__ rec,
                                                    dg2p_monitors* mon, long long blk) {
  __shared__ double sh[WT / 64];
  for (long long s = R_AMIN + blk; s < R_INT + 8; s += A.nblocks) {
    const int slot = (int)s;
    const double id = rec_identity(slot);
    double v[FUSED_RATE_PER_THREAD];
#pragma unroll
    for (int u = 0; u < FUSED_RATE_PER_THREAD; ++u) {
      const long long r = threadIdx.x + u * WT;
      v[u] = r < A.nrate ? rec[r * REC + slot] : id;
    }
    double acc = id;
#pragma unroll
    for (int u = 0; u < FUSED_RATE_PER_THREAD; ++u) acc = rec_combine(slot, acc, v[u]);
    acc = rec_wave(slot, acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double x = sh[0];
#pragma unroll
      for (int i = 1; i < WT / 64; ++i) x = rec_combine(slot, x, sh[i]);
      if (slot == R_AMIN) mon->min_alpha = x;
      else if (slot == R_AMAX) mon->max_alpha = x;
      else if (slot == R_BAD) mon->nonphys = (long long)x;
      else if (slot == R_DEVP) mon->dev_p = x;
      else if (slot == R_DEVU) mon->dev_u = x;
      else mon->integral[slot - R_INT] = slot - R_INT < NF ? x : 0.0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Stage pass: residual of each element (volume terms, sources, all faces, SIPG
// symmetric term), then MODE 0: store R; MODE 1: U_out = U_s + dt R;
// MODE 2: U_out = rk_a U_n + rk_b (U_s + dt R).  Epilogue on U_out: EPI = 1
// face ingredients into Gout, EPI = 2 also the reduction records.  BCK: 0 =
// periodic mesh (no ghost code), 1 = walls / extrapolation, 2 = also kinds
// that read the side's bc_state (Dirichlet, Riemann).
template <int DIM, bool VISC, bool CSF, int BCK, int MODE, int EPI, int PR>
__global__ __launch_bounds__(ewg<DIM>(), (min_waves<DIM, VISC>())) void k_stage(KArgs A, StageIO io) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  constexpr int NC = DIM + 3;  // conservative equations
  const long long blk = logical_block(A);
  if (blk < 0) return;
  const int lane = threadIdx.x & 63;
  // the wave's index in the workgroup, uniform by construction: read through
  // readfirstlane so that for hexahedra (one element per wave) the element,
  // its grid coordinates, neighbours and boundary tests are scalar values
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  constexpr int WT = ewg<DIM>();
  // element and its multi-index (hexahedra: one per workgroup, in the tiled
  // traversal order)
  long long ec[3] = {0, 0, 0};
  bool valid;
  long long e;
  if constexpr (DIM == 3) {
    static_assert(WT == 64 && EPW == 1, "one hexahedron per workgroup");
    tiled_coords(A, (unsigned)blk, ec);
    valid = true;
    e = ec[0] + A.N[0] * (ec[1] + (long long)A.N[1] * ec[2]);
  } else {
    const long long e0 = (blk * (WT / 64) + wv) * EPW + lane / NN;
    valid = e0 < A.E;
    e = valid ? e0 : A.E - 1;
    elem_coords<DIM>(A, e, ec);
  }
  const int node = lane % NN;
  int ak[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) ak[k] = (node >> (2 * k)) & 3;
  Deriv<DIM, PR> L;
  deriv_setup<DIM, PR>(A, ak, L);

  const double* __restrict__ Us = io.Us;
  double q[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) q[f] = Us[(f * A.E + e) * NN + node];
  // the step's dt (written before this launch), loaded now rather than at
  // the combine, where its wait would stall the wave
  double dt_in = 0.0;
  if constexpr (MODE != 0) {
    if (!(MODE == 1 && io.dt_out)) dt_in = *io.dt;
  }
  // first stage of a small grid: the rate records of the time step
  __shared__ double dt_lds[2][WT / 64];
  if constexpr (MODE == 1) {
    if (io.dt_out && (!io.dt_fixed || io.mon_out)) fused_dt_load<WT>(A, io.rate_in, dt_lds);
  }
  // face neighbours
  long long enb[DIM];
  bool bndk[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int akk = ak[k];
    const bool isface = (akk == 0) || (akk == 3);
    const int side = akk == 3;
    long long c = ec[k] + (side ? 1 : -1);
    bool bnd = false;
    if (c < 0 || c >= A.N[k]) {
      if (BCK == 0 || bc_kind(A, k, side) == DG2P_BC_PERIODIC)
        c = (c < 0) ? A.N[k] - 1 : 0;
      else
        bnd = true;
    }
    long long estr = 1;
#pragma unroll
    for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
    enb[k] = (isface && !bnd) ? e + (c - ec[k]) * estr : e;
    bndk[k] = bnd;
  }
  // 2D and 3D: the lane's face job (one x- or y-face node of its quad, or of
  // its z-layer of the hexahedron, see the face pass) and the neighbour trace
  // across it, loaded here so that the loads are in flight during the volume
  // terms.
  bool xjob = false, jbnd = false;
  int jside = 0, onode = 0;
  double qn[NF], an = 0.0, tn[DIM];
  if constexpr (DIM >= 2) {
    xjob = (ak[0] == 0) || (ak[0] == 3);
    jside = xjob ? (ak[0] == 3) : (ak[0] == 2);
    onode = xjob ? node : (DIM == 3 ? (node & ~15) : 0) + ak[1] + (jside ? 12 : 0);
    long long en;
    if (xjob) {
      en = enb[0];
      jbnd = bndk[0];
    } else {
      long long c = ec[1] + (jside ? 1 : -1);
      if (c < 0 || c >= A.N[1]) {
        if (BCK == 0 || bc_kind(A, 1, jside) == DG2P_BC_PERIODIC)
          c = (c < 0) ? A.N[1] - 1 : 0;
        else
          jbnd = true;
      }
      en = jbnd ? e : e + (c - ec[1]) * A.N[0];
    }
    const int nodee = xjob ? node + (3 - 2 * ak[0]) : onode + (jside ? -12 : 12);
    const int fn = DIM == 2 ? (xjob ? (node >> 2) : ak[1]) : (xjob ? face_index(node, 0) : face_index(onode, 1));
    face_load<DIM, VISC>(A, Us, io.Gin, xjob ? 0 : 1, jside, en, nodee, fn, qn, an, tn);
    // issue these loads before the closure waits for the element's own state
    // (the scheduler would otherwise place them behind it)
    if constexpr (DIM == 3) __builtin_amdgcn_sched_barrier(0);
  }
  Prim pr;
  closure<DIM>(A, q, pr);
  Grad<DIM, VISC> g;
  gradients<DIM, VISC, PR>(A, q, pr, L, g);
  double R[NF];
  // volume terms, strong form: R_q = sum_k (1/J_k) D_k (-F_q + s_q a + V_q)_k
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) {
    const double sq = s_coef<DIM>(A, pr, qi);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double fl = fma(sq, g.a[k], -conv_flux<DIM>(q, pr, qi, k));
      if constexpr (VISC) {
        if (qi >= 2 && qi < 2 + DIM) {
          fl = fma(g.mu, g.S[qi - 2][k], fl);
        } else if (qi == 2 + DIM) {
          double tu = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) tu = fma(g.S[j][k], pr.u[j], tu);
          fl = fma(g.mu, tu, fl);
        }
      }
      acc += dkp<DIM, PR>(fl, k, L, A);
    }
    R[qi] = acc;
  }
  {
    double acc = 0.0, ua = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      acc += dkp<DIM, PR>(g.a[k], k, L, A);
      ua = fma(pr.u[k], g.gA[k], ua);
    }
    R[3 + DIM] = acc - ua;  // div a, and transport as a volume source
    R[4 + DIM] = -g.upsi;
  }
  // sources: gravity and CSF surface tension
  {
    double csf = 0.0;
    if constexpr (CSF) {
      double div = 0.0, ga2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        div += dkp<DIM, PR>(g.nh[k], k, L, A);
        ga2 = fma(g.gA[k], g.gA[k], ga2);
      }
      const double kappa = -div;
      const double dG = sqrt_nr(ga2 + A.delta * A.delta) - A.delta;
      csf = A.sigma * kappa * dG;
    }
    if (A.has_grav || CSF) {
      double ew = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        double sj = pr.rho * A.grav[j];
        double ej = pr.rho * A.grav[j] * pr.u[j];
        if constexpr (CSF) {
          sj += csf * g.nh[j];
          ej += csf * pr.u[j] * g.nh[j];
        }
        R[2 + j] += sj;
        ew += ej;
      }
      R[2 + DIM] += ew;
    }
  }

  // Pin the volume and source sums here: otherwise their multiply-adds are
  // sunk past the face code while the lane rotations feeding them stay
  // behind, and the rotated values are spilled.
#pragma unroll
  for (int f = 0; f < NF; ++f) DG2P_PIN(R[f]);

  // faces
  const double* __restrict__ Gin = io.Gin;
  // hexahedra: the z-face neighbour traces, loaded by the z-face lanes before
  // the x/y faces are evaluated, so that they are in flight meanwhile
  double qz[NF], anz = 0.0, tz[DIM];
  if constexpr (DIM == 3) {
    const int akz = ak[2];
    if (akz == 0 || akz == 3)
      face_load<DIM, VISC>(A, Us, Gin, 2, akz == 3, enb[2], node + (3 - 2 * akz) * 16, face_index(node, 2), qz, anz,
                           tz);
  }
  if constexpr (DIM >= 2) {
    // The 16 x- and y-face nodes of a quad (4 faces x 4 nodes), or of one
    // z-layer of a hexahedron, are spread over its 16 lanes, one face
    // evaluation each: a lane with a_x in {0, 3} evaluates the x-face at its
    // own node; a lane with a_x = 1 (2) evaluates the low (high) y-face at
    // node (a_y, 0, a_z) ((a_y, 3, a_z)).  The owner node's trace comes from
    // its lane and the results go back to it by lane exchanges, so no x or y
    // face is evaluated on half-idle lanes; the z-faces of a hexahedron
    // follow as in the loop form.
    const int olane = (lane & 48) | (DIM == 2 ? onode : (onode & 15));
    double qo[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) qo[f] = __shfl(q[f], olane);
    Prim po;
    po.rho = __shfl(pr.rho, olane);
    po.u[0] = __shfl(pr.u[0], olane);
    po.u[1] = __shfl(pr.u[1], olane);
    po.u[2] = DIM == 3 ? __shfl(pr.u[2], olane) : 0.0;
    po.kin = __shfl(pr.kin, olane);
    po.P = __shfl(pr.P, olane);
    po.c = __shfl(pr.c, olane);
    po.sE = __shfl(pr.sE, olane);
    const double a1 = __shfl(g.a[1], olane);
    const double ao = xjob ? g.a[0] : a1;
    double mu = 0.0, Sk[DIM] = {};
    if constexpr (VISC && DIM == 2) {
      const double mu1 = __shfl(g.mu, olane), s01 = __shfl(g.S[0][1], olane), s11 = __shfl(g.S[1][1], olane);
      mu = xjob ? g.mu : mu1;
      Sk[0] = xjob ? g.S[0][0] : s01;
      Sk[1] = xjob ? g.S[1][0] : s11;
    } else if constexpr (VISC) {
      const double mu1 = __shfl(g.mu, olane);
      mu = xjob ? g.mu : mu1;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const double sj1 = __shfl(g.S[j][1], olane);
        Sk[j] = xjob ? g.S[j][0] : sj1;
      }
    }
    double gAk = 0.0, nhk = 0.0;
    if constexpr (BCK == 2) {
      const double ga1 = __shfl(g.gA[1], olane), nh1 = __shfl(g.nh[1], olane);
      gAk = xjob ? g.gA[0] : ga1;
      nhk = xjob ? g.nh[0] : nh1;
    }
    double Rc[NF], sv[NC + 1];
    face_flux<DIM, VISC, BCK>(A, xjob ? 0 : 1, jside, jbnd, qn, an, tn, qo, po, ao, mu, Sk, gAk, nhk, Rc, sv);
    double symv[NC + 1];
#pragma unroll
    for (int i = 0; i <= NC; ++i) symv[i] = xjob ? sv[i] : 0.0;
    if (xjob) {
#pragma unroll
      for (int f = 0; f < NF; ++f) R[f] += Rc[f];
    }
    spread_sym<0, DIM>(A, ak[0], symv, R);
    // y-face results of this lane's node, from the lane that evaluated them
    const bool yown = (ak[1] == 0) || (ak[1] == 3);
    const int jl = (lane & 48) | ((ak[1] == 3 ? 2 : 1) + 4 * ak[0]);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double r = __shfl(Rc[f], jl);
      if (yown) R[f] += r;
    }
#pragma unroll
    for (int i = 0; i <= NC; ++i) {
      const double v = __shfl(sv[i], jl);
      symv[i] = yown ? v : 0.0;
    }
    spread_sym<(DIM > 1 ? 1 : 0), DIM>(A, ak[1], symv, R);
  }
  // hexahedra, later stages: U^n of the stage combination, loaded now so that
  // the loads are in flight during the z-faces
  [[maybe_unused]] double unr[NF];
  if constexpr (DIM == 3 && MODE == 2) {
#pragma unroll
    for (int f = 0; f < NF; ++f) unr[f] = __builtin_nontemporal_load(&io.Un[(f * A.E + e) * NN + node]);
  }
  {
    // 1D: its faces; 3D: the z-faces (lanes with a_z in {0, 3})
    constexpr int K0 = DIM >= 2 ? 2 : 0;
#pragma unroll
    for (int k = K0; k < DIM; ++k) {
      const int S = 1 << (2 * k);
      const int akk = ak[k];
      double symv[NC + 1];
#pragma unroll
      for (int i = 0; i <= NC; ++i) symv[i] = 0.0;
      if ((akk == 0) || (akk == 3)) {
        double Rc[NF], Sk[DIM];
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          if constexpr (VISC) Sk[j] = g.S[j][k];
          else Sk[j] = 0.0;
        }
        double gAk = 0.0, nhk = 0.0;
        if constexpr (BCK == 2) {
          gAk = g.gA[k];
          nhk = g.nh[k];
        }
        double qk[NF], ank, tk[DIM];
        if constexpr (DIM == 3) {
#pragma unroll
          for (int f = 0; f < NF; ++f) qk[f] = qz[f];
          ank = anz;
#pragma unroll
          for (int j = 0; j < DIM; ++j) tk[j] = tz[j];
        } else {
          face_load<DIM, VISC>(A, Us, Gin, k, akk == 3, enb[k], node + (3 - 2 * akk) * S, face_index(node, k), qk,
                               ank, tk);
        }
        face_flux<DIM, VISC, BCK>(A, k, akk == 3, bndk[k], qk, ank, tk, q, pr, g.a[k], g.mu, Sk, gAk, nhk, Rc, symv);
#pragma unroll
        for (int f = 0; f < NF; ++f) R[f] += Rc[f];
      }
      if (k == 0) spread_sym<0, DIM>(A, akk, symv, R);
      else if (k == 1) spread_sym<(DIM > 1 ? 1 : 0), DIM>(A, akk, symv, R);
      else spread_sym<(DIM > 2 ? 2 : 0), DIM>(A, akk, symv, R);
    }
  }

  // the fused time step of a small grid (uniform branch), needed from here on
  double dt_fused = 0.0;
  if constexpr (MODE == 1) {
    if (io.dt_out) {
      double rate = 0.0;
      if (!io.dt_fixed || io.mon_out) rate = fused_rate_finish<WT>(A, dt_lds, 16.0 * DIM);
      dt_fused = io.dt_fixed ? *io.dt_fixed : A.cfl / rate;
      if (blk == 0 && threadIdx.x == 0) {
        *io.dt_out = dt_fused;
        if (io.t) *io.t += dt_fused;
        if (io.mon_out) {
          io.mon_out->max_rate = rate;
          io.mon_out->dt = dt_fused;
        }
      }
    }
  }
  const long long o = e * NN + node;
  const long long fs = A.E * NN;
  if constexpr (MODE == 0) {
    if (valid) {
#pragma unroll
      for (int f = 0; f < NF; ++f) io.Out[f * fs + o] = R[f];
    }
  } else {
    const double dt = (MODE == 1 && io.dt_out) ? dt_fused : dt_in;
    // the combination with explicit fused multiply-adds, so that every
    // variant of the kernel (with or without records) rounds it the same way
    double uo[NF];
    if constexpr (MODE == 1) {
#pragma unroll
      for (int f = 0; f < NF; ++f) uo[f] = fma(dt, R[f], q[f]);
    } else if constexpr (DIM == 3) {
#pragma unroll
      for (int f = 0; f < NF; ++f) uo[f] = fma(A.rk_a, unr[f], A.rk_b * fma(dt, R[f], q[f]));
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) uo[f] = fma(A.rk_a, io.Un[f * fs + o], A.rk_b * fma(dt, R[f], q[f]));
    }
    if (valid) {
#pragma unroll
      for (int f = 0; f < NF; ++f) store_out<DIM>(&io.Out[f * fs + o], uo[f]);
    }
    if constexpr (EPI > 0)
      emit<DIM, VISC, true, (EPI == 2 ? 2 : (EPI == 3 ? 1 : 0)), PR>(A, uo, e, valid, node, ak, L, io.Gout, io.rec,
                                                                   blk, io.rate_out);
    if constexpr (MODE == 1) {
      if (io.mon_out) fused_monitor_slots<WT, NF>(A, io.mon_rec, io.mon_out, blk);
    }
  }
}

// ---------------------------------------------------------------------------
// Initial-condition map (primitive -> conserved), one thread per node.
template <int DIM>
__global__ void k_prim_to_cons(KArgs A, const double* __restrict__ P, double* __restrict__ U,
                               long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double al = P[0 * n + i], ps = P[1 * n + i], r1 = P[2 * n + i], r2 = P[3 * n + i];
  const double p = P[(4 + DIM) * n + i];
  const double q1 = al * r1, q2 = (1.0 - al) * r2;
  const double rho = q1 + q2;
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
  double k2 = 0.0;
  U[0 * n + i] = q1;
  U[1 * n + i] = q2;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double u = P[(4 + j) * n + i];
    k2 = fma(u, u, k2);
    U[(2 + j) * n + i] = rho * u;
  }
  U[(2 + DIM) * n + i] = xi * p + pi + rho * (0.5 * k2);
  U[(3 + DIM) * n + i] = al;
  U[(4 + DIM) * n + i] = ps;
}

// Reverse of the initial-condition map: primitive cotangents from U_bar.
template <int DIM>
__global__ void k_prim_to_cons_vjp(KArgs A, const double* __restrict__ P, const double* __restrict__ Ub,
                                   double* __restrict__ Pb, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double al = P[0 * n + i], r1 = P[2 * n + i], r2 = P[3 * n + i];
  const double p = P[(4 + DIM) * n + i];
  const double rho = al * r1 + (1.0 - al) * r2;
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  double k2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double u = P[(4 + j) * n + i];
    k2 = fma(u, u, k2);
  }
  const double Eb = Ub[(2 + DIM) * n + i];
  // rho E = xi P + Pi + rho k
  double rhob = 0.5 * k2 * Eb;
  const double xib = p * Eb, pib = Eb;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double u = P[(4 + j) * n + i];
    const double mb = Ub[(2 + j) * n + i];
    rhob += u * mb;
    Pb[(4 + j) * n + i] = rho * mb + rho * u * Eb;
  }
  Pb[(4 + DIM) * n + i] = xi * Eb;
  const double q1b = Ub[0 * n + i] + rhob, q2b = Ub[1 * n + i] + rhob;
  Pb[0 * n + i] = r1 * q1b - r2 * q2b + (A.xi1 - A.xi2) * xib + (A.pi1 - A.pi2) * pib + Ub[(3 + DIM) * n + i];
  Pb[1 * n + i] = Ub[(4 + DIM) * n + i];
  Pb[2 * n + i] = al * q1b;
  Pb[3 * n + i] = (1.0 - al) * q2b;
}

// ---------------------------------------------------------------------------
// Records of a state without face ingredients (dt / monitor requests):
// grid-stride over nodes, fixed grid.
template <int DIM, bool VISC>
__global__ __launch_bounds__(BLOCK) void k_records(KArgs A, const double* __restrict__ U,
                                                   double* __restrict__ rec) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int NF = DIM + 5;
  const long long n = A.E * NN;
  double acc[REC];
#pragma unroll
  for (int s = 0; s < REC; ++s) acc[s] = (s == R_AMIN) ? INFINITY : (s == R_AMAX ? -INFINITY : 0.0);
  // the loop bound depends on the workgroup only, so every thread reaches the reduction
  for (long long base = (long long)blockIdx.x * BLOCK; base < n; base += (long long)gridDim.x * BLOCK) {
    const long long i = base + threadIdx.x;
    const bool valid = i < n;
    const long long ii = valid ? i : 0;
    double q[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) q[f] = U[f * n + ii];
    Prim p;
    closure<DIM>(A, q, p);
    double v[REC];
    node_record<DIM, VISC>(A, q, p, (int)(ii % NN), valid, v);
#pragma unroll
    for (int s = 0; s < REC; ++s) acc[s] = rec_combine(s, acc[s], v[s]);
  }
  block_record(acc, rec, blockIdx.x);
}

// Records are reduced with one slot per thread: thread t of a workgroup of NT
// threads reads slot t mod REC of records lo + t / REC, lo + t / REC + NT / REC,
// ... (contiguous loads), then threads holding the same slot are combined
// (lanes 16 and 32 apart in the wave, then the waves through LDS).  The
// combination order is fixed, so the result is deterministic.
template <int NS, int NT>
__device__ __forceinline__ void reduce_slots(const double* __restrict__ rec, long long lo, long long hi,
                                             double* red) {
  static_assert(NT % 64 == 0 && 64 % NS == 0, "slot-per-thread layout");
  const int s = threadIdx.x % NS;
  const double id = rec_identity(s);
  double acc = id;
  // batches of RB independent loads in flight (the records come from other
  // XCDs' caches, so each load is a long-latency trip), combined in order
  constexpr int RB = 8;
  constexpr long long ST = NT / NS;
  for (long long r0 = lo + threadIdx.x / NS; r0 < hi; r0 += RB * ST) {
    double v[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const long long r = r0 + u * ST;
      v[u] = r < hi ? rec[r * NS + s] : id;
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) acc = rec_combine(s, acc, v[u]);
  }
#pragma unroll
  for (int m = NS; m < 64; m <<= 1) acc = rec_combine(s, acc, __shfl_xor(acc, m));
  __shared__ double sh[NT / 64][NS];
  if ((threadIdx.x & 63) < NS) sh[threadIdx.x >> 6][s] = acc;
  __syncthreads();
  if (threadIdx.x < NS) {
    double x = sh[0][s];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) x = rec_combine(s, x, sh[i][s]);
    red[s] = x;
  }
}

// First-level reduction of records of NS slots: workgroup j combines records
// [j*chunk, min((j+1)*chunk, n)) into record j of out.
template <int NS>
__global__ __launch_bounds__(BLOCK) void k_reduce_records(const double* __restrict__ rec, long long n,
                                                          long long chunk, double* __restrict__ out) {
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  __shared__ double red[NS];
  reduce_slots<NS, BLOCK>(rec, lo, hi, red);
  __syncthreads();
  if (threadIdx.x < NS) out[(long long)blockIdx.x * NS + threadIdx.x] = red[threadIdx.x];
}

// Final reduction: time-step rule and monitors.  rate = (max wave + (p+1)^2 d
// nu_max / h_min) / h_min with nu_max = max(Gamma eps, max mu/rho); dt = cfl / rate.
// One workgroup of FIN_THREADS threads.
constexpr int FIN_THREADS = 1024;
static __global__ __attribute__((unused)) __launch_bounds__(FIN_THREADS) void k_finalize(const double* __restrict__ rec, long long n,
                                                          double GammaEps, double pdim, int nf, double hmin,
                                                          double cfl, const double* dt_fixed, double* dt,
                                                          double* t, dg2p_monitors* mon) {
  __shared__ double red[REC];
  reduce_slots<REC, FIN_THREADS>(rec, 0, n, red);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rate = rate_of(red[R_WAVE], red[R_NU], GammaEps, pdim, hmin);
    const double d = dt_fixed ? *dt_fixed : cfl / rate;
    if (dt) *dt = d;
    if (t) *t += d;
    if (mon) {
      mon->max_rate = rate;
      mon->dt = d;
      mon->min_alpha = red[R_AMIN];
      mon->max_alpha = red[R_AMAX];
      for (int f = 0; f < 8; ++f) mon->integral[f] = f < nf ? red[R_INT + f] : 0.0;
      mon->dev_p = red[R_DEVP];
      mon->dev_u = red[R_DEVU];
      mon->nonphys = (long long)red[R_BAD];
    }
  }
}

// Final reduction of rate records (time step only): *dt = cfl / rate (or
// *dt_fixed), *t += dt.
static __global__ __attribute__((unused)) __launch_bounds__(FIN_THREADS) void k_finalize_rate(const double* __restrict__ rec, long long n,
                                                               double GammaEps, double pdim, double hmin, double cfl,
                                                               const double* dt_fixed, double* dt, double* t) {
  __shared__ double red[RATE];
  reduce_slots<RATE, FIN_THREADS>(rec, 0, n, red);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double d = dt_fixed ? *dt_fixed : cfl / rate_of(red[R_WAVE], red[R_NU], GammaEps, pdim, hmin);
    *dt = d;
    if (t) *t += d;
  }
}

}  // namespace dg2p
