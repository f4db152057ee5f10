// Device side of libdg2p: HIP kernels for gfx950 (wave64).
//
// Mapping: one lane per GLL node.  An element of 4^d nodes occupies 4^d
// consecutive lanes (1D: 4 lanes, 16 elements per wave; 2D: 16 lanes, 4
// elements per wave; 3D: the whole 64-lane wave), so a wave-wide load of one
// field of U[f][e][j] is 512 contiguous bytes.  The lane index inside an
// element is the node index j = a_x + 4 a_y + 16 a_z, so the nodes of a line
// along axis k sit at lane stride 4^k, and the 4-point derivative contraction
// along k is a cross-lane gather inside the wave (no LDS round trip).
//
// Every element evaluates all of its own faces ("owner computes"): the
// numerical fluxes are recomputed from both traces by the two elements that
// share a face, so no face buffer is ever written twice and the result is
// deterministic without atomics.  The neighbour's normal interface flux
// a.e_k and viscous traction tau.e_k at its face nodes need its own
// element-local gradients; they are produced by a separate pass
// (face-ingredient buffer G) because a neighbour's gradient needs the whole
// neighbour element.

#pragma once

#include <hip/hip_runtime.h>

#include "../../include/dg2p.h"

namespace dg2p {

constexpr int NP = 4;  // GLL nodes per axis (p = 3)

struct KArgs {
  long long E;
  int N[3];
  int bc[3][2];
  double bcs[3][2][8];
  double Jinv[3];
  double lift[3];       // 1 / (w_0 J_k): face-to-node lift under GLL collocation
  double pen[3];        // c_ip (p+1)^2 / h_k
  double D[4][4];       // D[a][b] = l_b'(xi_a)
  double symw[3][2][4]; // D[end][a] / (2 w_a J_k^2), end = 0 (low side) or 3 (high side)
  double wJ[3][4];      // w_a J_k (diagonal mass factors)
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
};

struct Prim {
  double rho, u[3], kin, P, c, rH1, rH2;
};

__device__ __forceinline__ double sel4(int a, double c0, double c1, double c2, double c3) {
  return a == 0 ? c0 : (a == 1 ? c1 : (a == 2 ? c2 : c3));
}

// Stiffened-gas primitive recovery of one node (closure of the five-equation
// model): P = (rho e - Pi) / xi with the mixture xi = sum alpha_l/(gamma_l-1)
// and Pi = sum alpha_l gamma_l Pinf_l/(gamma_l-1); frozen mixture sound speed
// c^2 = ((1+xi) P + Pi) / (xi rho); rho_l H_l = gamma_l (P + Pinf_l)/(gamma_l-1).
template <int DIM>
__device__ __forceinline__ void closure(const KArgs& A, const double* q, Prim& p) {
  p.rho = q[0] + q[1];
  double k2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    p.u[j] = q[2 + j] / p.rho;
    k2 = fma(p.u[j], p.u[j], k2);
  }
  p.kin = 0.5 * k2;
  const double al = q[3 + DIM];
  const double rhoe = q[2 + DIM] - p.rho * p.kin;
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
  p.P = (rhoe - pi) / xi;
  p.c = sqrt(((1.0 + xi) * p.P + pi) / (xi * p.rho));
  p.rH1 = A.gh1 * (p.P + A.pinf1);
  p.rH2 = A.gh2 * (p.P + A.pinf2);
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
  return dr * p.kin + p.rH1 - p.rH2;
}

// Convective flux of conservative equation q along axis k.
template <int DIM>
__device__ __forceinline__ double conv_flux(const double* q, const Prim& p, int qi, int k) {
  if (qi < 2) return q[qi] * p.u[k];
  if (qi < 2 + DIM) return q[qi] * p.u[k] + ((qi - 2) == k ? p.P : 0.0);
  return (q[2 + DIM] + p.P) * p.u[k];
}

// 4-point derivative contraction along the lane stride S = 4^k:
// sum_b D[a_k][b] f(.., b, ..); Dr = row a_k of D.
__device__ __forceinline__ double contract(double f, int lane, int ak, int S, const double* Dr) {
  const int base = lane - ak * S;
  double r = Dr[0] * __shfl(f, base);
  r = fma(Dr[1], __shfl(f, base + S), r);
  r = fma(Dr[2], __shfl(f, base + 2 * S), r);
  r = fma(Dr[3], __shfl(f, base + 3 * S), r);
  return r;
}

// Index of a node inside the face layer normal to axis k (axis k removed).
__device__ __forceinline__ int face_index(int node, int k) {
  const int lowmask = (1 << (2 * k)) - 1;
  return (node & lowmask) | ((node >> (2 * k + 2)) << (2 * k));
}

// Per-lane element-local quantities shared by the ingredient and stage passes.
template <int DIM, bool VISC>
struct NodeState {
  static constexpr int NF = DIM + 5;
  double q[NF];
  Prim pr;
  double gA[DIM], gP[DIM], nh[DIM], a[DIM];
  double S[VISC ? DIM : 1][VISC ? DIM : 1];  // grad u + grad u^T - 2/3 div u I
  double mu;
};

template <int DIM, bool VISC>
__device__ __forceinline__ void element_quantities(const KArgs& A, NodeState<DIM, VISC>& s,
                                                   int lane, const int* ak,
                                                   const double (*Dr)[4]) {
  closure<DIM>(A, s.q, s.pr);
  const double al = s.q[3 + DIM];
  const double ps = s.q[4 + DIM];
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int S = 1 << (2 * k);
    s.gA[k] = contract(al, lane, ak[k], S, Dr[k]) * A.Jinv[k];
    s.gP[k] = contract(ps, lane, ak[k], S, Dr[k]) * A.Jinv[k];
    g2 = fma(s.gP[k], s.gP[k], g2);
  }
  const double nrm = sqrt(g2 + A.delta * A.delta);
  const double aa = al * (1.0 - al);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    s.nh[k] = s.gP[k] / nrm;
    s.a[k] = A.Gamma * (A.eps * s.gA[k] - aa * s.nh[k]);
  }
  if constexpr (VISC) {
    double gU[DIM][DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k)
        gU[j][k] = contract(s.pr.u[j], lane, ak[k], 1 << (2 * k), Dr[k]) * A.Jinv[k];
    double div = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) div += gU[j][j];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k)
        s.S[j][k] = gU[j][k] + gU[k][j] - (j == k ? (2.0 / 3.0) * div : 0.0);
    s.mu = A.mu1 * al + A.mu2 * (1.0 - al);
  } else {
    s.mu = 0.0;
  }
}

template <int DIM>
__device__ __forceinline__ void lane_setup(const KArgs& A, int node, int* ak, double (*Dr)[4]) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    ak[k] = (node >> (2 * k)) & 3;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      Dr[k][b] = sel4(ak[k], A.D[0][b], A.D[1][b], A.D[2][b], A.D[3][b]);
  }
}

// ---------------------------------------------------------------------------
// Face-ingredient pass: for every element and each of its 2d faces, the
// normal component along +e_k of the interface flux a (and of the viscous
// stress tau[j][k]) at the face nodes.  G[((2k+side)*C + comp)*E + e][fn].
template <int DIM, bool VISC>
__global__ __launch_bounds__(64) void k_face_ingredients(KArgs A, const double* __restrict__ U,
                                                         double* __restrict__ G) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  constexpr int C = VISC ? 1 + DIM : 1;
  constexpr int NFN = NN / 4;
  const int lane = threadIdx.x;
  const long long e0 = (long long)blockIdx.x * EPW + lane / NN;
  const bool valid = e0 < A.E;
  const long long e = valid ? e0 : A.E - 1;
  const int node = lane % NN;
  int ak[3];
  double Dr[3][4];
  lane_setup<DIM>(A, node, ak, Dr);
  NodeState<DIM, VISC> s;
#pragma unroll
  for (int f = 0; f < NF; ++f) s.q[f] = U[(f * A.E + e) * NN + node];
  element_quantities<DIM, VISC>(A, s, lane, ak, Dr);
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (ak[k] != 0 && ak[k] != 3) continue;
    const int side = ak[k] == 3;
    const int fn = face_index(node, k);
    const long long base = (long long)((2 * k + side) * C) * A.E;
    G[(base + e) * NFN + fn] = s.a[k];
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) G[(base + (long long)(1 + j) * A.E + e) * NFN + fn] = s.mu * s.S[j][k];
    }
  }
}

// ---------------------------------------------------------------------------
// Stage pass: residual of one element (volume terms, sources, all faces,
// SIPG symmetric term), then either R is stored (MODE 0), or the RK stage
// U_out = U_s + dt R (MODE 1), or U_out = rk_a U_n + rk_b (U_s + dt R) (MODE 2).
template <int DIM, bool VISC, bool CSF, int MODE>
__global__ __launch_bounds__(64) void k_stage(KArgs A, const double* __restrict__ Us,
                                              const double* __restrict__ G,
                                              const double* Un, double* Out,
                                              const double* __restrict__ dtp) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  constexpr int NC = DIM + 3;  // conservative equations
  constexpr int C = VISC ? 1 + DIM : 1;
  constexpr int NFN = NN / 4;
  const int lane = threadIdx.x;
  const long long e0 = (long long)blockIdx.x * EPW + lane / NN;
  const bool valid = e0 < A.E;
  const long long e = valid ? e0 : A.E - 1;
  const int node = lane % NN;
  int ak[3];
  double Dr[3][4];
  lane_setup<DIM>(A, node, ak, Dr);

  NodeState<DIM, VISC> s;
#pragma unroll
  for (int f = 0; f < NF; ++f) s.q[f] = Us[(f * A.E + e) * NN + node];
  element_quantities<DIM, VISC>(A, s, lane, ak, Dr);
  const double* q = s.q;
  const Prim& pr = s.pr;

  double R[NF];
  // volume terms, strong form: R_q = sum_k (1/J_k) D_k (-F_q + s_q a + V_q)_k
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) {
    const double sq = s_coef<DIM>(A, pr, qi);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double fl = -conv_flux<DIM>(q, pr, qi, k) + sq * s.a[k];
      if constexpr (VISC) {
        if (qi >= 2 && qi < 2 + DIM) {
          fl += s.mu * s.S[qi - 2][k];
        } else if (qi == 2 + DIM) {
          double tu = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) tu = fma(s.S[j][k], pr.u[j], tu);
          fl += s.mu * tu;
        }
      }
      acc += contract(fl, lane, ak[k], 1 << (2 * k), Dr[k]) * A.Jinv[k];
    }
    R[qi] = acc;
  }
  {
    double acc = 0.0, ua = 0.0, up = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      acc += contract(s.a[k], lane, ak[k], 1 << (2 * k), Dr[k]) * A.Jinv[k];
      ua = fma(pr.u[k], s.gA[k], ua);
      up = fma(pr.u[k], s.gP[k], up);
    }
    R[3 + DIM] = -ua + acc;  // transport as a volume source + div a
    R[4 + DIM] = -up;
  }
  // sources: gravity and CSF surface tension
  {
    double csf = 0.0;
    if constexpr (CSF) {
      double div = 0.0, ga2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        div += contract(s.nh[k], lane, ak[k], 1 << (2 * k), Dr[k]) * A.Jinv[k];
        ga2 = fma(s.gA[k], s.gA[k], ga2);
      }
      const double kappa = -div;
      const double dG = sqrt(ga2 + A.delta * A.delta) - A.delta;
      csf = A.sigma * kappa * dG;
    }
    if (A.has_grav || CSF) {
      double ew = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        double sj = pr.rho * A.grav[j];
        double ej = pr.rho * A.grav[j] * pr.u[j];
        if constexpr (CSF) {
          sj += csf * s.nh[j];
          ej += csf * pr.u[j] * s.nh[j];
        }
        R[2 + j] += sj;
        ew += ej;
      }
      R[2 + DIM] += ew;
    }
  }

  // faces
  long long ec[3];
  {
    long long r = e;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      ec[k] = r % A.N[k];
      r /= A.N[k];
    }
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int S = 1 << (2 * k);
    const int akk = ak[k];
    const bool isface = (akk == 0) || (akk == 3);
    double symv[NC + 1];
#pragma unroll
    for (int i = 0; i <= NC; ++i) symv[i] = 0.0;
    if (isface) {
      const int side = akk == 3;
      const double sm = side ? 1.0 : -1.0;
      long long c = ec[k] + (side ? 1 : -1);
      bool bnd = false;
      if (c < 0 || c >= A.N[k]) {
        if (A.bc[k][side] == DG2P_BC_PERIODIC)
          c = (c < 0) ? A.N[k] - 1 : 0;
        else
          bnd = true;
      }
      double qe[NF];
      double aek;
      double tek[DIM];
      if (!bnd) {
        long long estr = 1;
#pragma unroll
        for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
        const long long en = e + (c - ec[k]) * estr;
        const int nodee = node + (3 - 2 * akk) * S;
#pragma unroll
        for (int f = 0; f < NF; ++f) qe[f] = Us[(f * A.E + en) * NN + nodee];
        const int fn = face_index(node, k);
        const long long gb = (long long)((2 * k + 1 - side) * C) * A.E;
        aek = G[(gb + en) * NFN + fn];
        if constexpr (VISC) {
#pragma unroll
          for (int j = 0; j < DIM; ++j) tek[j] = G[(gb + (long long)(1 + j) * A.E + en) * NFN + fn];
        }
      } else {
        const int kind = A.bc[k][side];
#pragma unroll
        for (int f = 0; f < NF; ++f) qe[f] = q[f];
        if (kind == DG2P_BC_SLIP_WALL) {
          qe[2 + k] = -q[2 + k];
          aek = -s.a[k];
          if constexpr (VISC) {
#pragma unroll
            for (int j = 0; j < DIM; ++j) tek[j] = (j == k ? 1.0 : -1.0) * (s.mu * s.S[j][k]);
          }
        } else if (kind == DG2P_BC_DIRICHLET) {
#pragma unroll
          for (int f = 0; f < 4 + DIM; ++f) qe[f] = A.bcs[k][side][f];
          const double ag = qe[3 + DIM];
          aek = A.Gamma * (A.eps * s.gA[k] - (ag * (1.0 - ag)) * s.nh[k]);
          if constexpr (VISC) {
            const double mug = A.mu1 * ag + A.mu2 * (1.0 - ag);
#pragma unroll
            for (int j = 0; j < DIM; ++j) tek[j] = mug * s.S[j][k];
          }
        } else {  // extrapolate
          aek = s.a[k];
          if constexpr (VISC) {
#pragma unroll
            for (int j = 0; j < DIM; ++j) tek[j] = s.mu * s.S[j][k];
          }
        }
      }
      Prim pe;
      closure<DIM>(A, qe, pe);
      const double umI = sm * pr.u[k], umE = sm * pe.u[k];
      const double lam = fmax(fabs(umI) + pr.c, fabs(umE) + pe.c);
      const double amI = sm * s.a[k], amE = sm * aek;
      const double alI = q[3 + DIM], alE = qe[3 + DIM];
      const double jump = alI - alE;
      const double ahat = 0.5 * (amI + amE) - A.pen[k] * A.GammaEps * jump;
      const double L = A.lift[k];
      double mue = 0.0, etav = 0.0;
      if constexpr (VISC) {
        mue = A.mu1 * alE + A.mu2 * (1.0 - alE);
        etav = A.pen[k] * (0.5 * (s.mu + mue));
      }
#pragma unroll
      for (int qi = 0; qi < NC; ++qi) {
        const double FmI = sm * conv_flux<DIM>(q, pr, qi, k);
        const double FmE = sm * conv_flux<DIM>(qe, pe, qi, k);
        const double Fhat = 0.5 * (FmI + FmE) - 0.5 * lam * (qe[qi] - q[qi]);
        const double sI = s_coef<DIM>(A, pr, qi), sE = s_coef<DIM>(A, pe, qi);
        const double sbar = 0.5 * (sI + sE);
        double t = (FmI - Fhat) + (sbar * ahat - sI * amI);
        if constexpr (VISC) {
          if (qi >= 2) {
            double VmI, VmE, pen;
            if (qi < 2 + DIM) {
              const int j = qi - 2;
              VmI = sm * (s.mu * s.S[j][k]);
              VmE = sm * tek[j];
              pen = etav * (pr.u[j] - pe.u[j]);
            } else {
              double tuI = 0.0, tuE = 0.0, du = 0.0;
#pragma unroll
              for (int j = 0; j < DIM; ++j) {
                tuI += (s.mu * s.S[j][k]) * pr.u[j];
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
        R[qi] += L * t;
        symv[qi] = sm * sbar * A.GammaEps * jump;
      }
      const double KA = 0.5 * (lam - umI) * (alE - alI);
      R[3 + DIM] += L * (KA + (ahat - amI));
      symv[NC] = sm * A.GammaEps * jump;
      R[4 + DIM] += L * (0.5 * (lam - umI) * (qe[4 + DIM] - q[4 + DIM]));
    }
    // SIPG symmetric term, spread along the normal line through each face node
    const int base = lane - akk * S;
    const double wlo = sel4(akk, A.symw[k][0][0], A.symw[k][0][1], A.symw[k][0][2], A.symw[k][0][3]);
    const double whi = sel4(akk, A.symw[k][1][0], A.symw[k][1][1], A.symw[k][1][2], A.symw[k][1][3]);
#pragma unroll
    for (int i = 0; i <= NC; ++i) {
      const double lo = __shfl(symv[i], base);
      const double hi = __shfl(symv[i], base + 3 * S);
      const int f = (i < NC) ? i : 3 + DIM;
      R[f] += lo * wlo + hi * whi;
    }
  }

  if (!valid) return;
  const long long o = e * NN + node;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f) Out[f * A.E * NN + o] = R[f];
  } else {
    const double dt = *dtp;
    if constexpr (MODE == 1) {
#pragma unroll
      for (int f = 0; f < NF; ++f) Out[f * A.E * NN + o] = q[f] + dt * R[f];
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double un = Un[f * A.E * NN + o];
        Out[f * A.E * NN + o] = A.rk_a * un + A.rk_b * (q[f] + dt * R[f]);
      }
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

// ---------------------------------------------------------------------------
// Reductions.  Block size 256, fixed grid (RED_BLOCKS), fixed order: the
// results are bitwise reproducible.
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;
constexpr int MON_SLOTS = 16;  // per-block partial record of the monitor pass

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int DIM, bool VISC>
__global__ __launch_bounds__(RED_THREADS) void k_rate_partial(KArgs A, const double* __restrict__ U,
                                                              double* __restrict__ part) {
  constexpr int NN = 1 << (2 * DIM);
  const long long n = A.E * NN;
  double mw = 0.0, mn = 0.0;
  for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * RED_THREADS) {
    double q[DIM + 5];
#pragma unroll
    for (int f = 0; f < DIM + 4; ++f) q[f] = U[f * n + i];
    q[DIM + 4] = 0.0;
    Prim p;
    closure<DIM>(A, q, p);
    double w = DIM * p.c;
#pragma unroll
    for (int j = 0; j < DIM; ++j) w += fabs(p.u[j]);
    mw = fmax(mw, w);
    if constexpr (VISC) {
      const double al = q[3 + DIM];
      mn = fmax(mn, (A.mu1 * al + A.mu2 * (1.0 - al)) / p.rho);
    }
  }
  __shared__ double sh[2][RED_THREADS / 64];
  mw = wave_max(mw);
  mn = wave_max(mn);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = mw;
    sh[1][threadIdx.x >> 6] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sh[0][0], b = sh[1][0];
    for (int i = 1; i < RED_THREADS / 64; ++i) {
      a = fmax(a, sh[0][i]);
      b = fmax(b, sh[1][i]);
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// nu_max = max(Gamma eps, max mu/rho); rate = (max wave + (p+1)^2 d nu_max / h_min) / h_min.
__global__ __launch_bounds__(RED_THREADS) void k_rate_final(const double* __restrict__ part, int nblk,
                                                            double GammaEps, int dim, double hmin,
                                                            double cfl, double* dt,
                                                            dg2p_monitors* mon) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += RED_THREADS) {
    a = fmax(a, part[2 * i]);
    b = fmax(b, part[2 * i + 1]);
  }
  __shared__ double sh[2][RED_THREADS / 64];
  a = wave_max(a);
  b = wave_max(b);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < RED_THREADS / 64; ++i) {
      sh[0][0] = fmax(sh[0][0], sh[0][i]);
      sh[1][0] = fmax(sh[1][0], sh[1][i]);
    }
    const double nu = fmax(GammaEps, sh[1][0]);
    const double rate = (sh[0][0] + 16.0 * dim * nu / hmin) / hmin;
    const double d = cfl / rate;
    if (dt) *dt = d;
    if (mon) {
      mon->max_rate = rate;
      mon->dt = d;
    }
  }
}

// Monitor partials per block: [0..NF) integrals, NF: min alpha, NF+1: max alpha,
// NF+2: max |P - p_ref|, NF+3: max |u - u_ref|, NF+4: non-physical count.
template <int DIM>
__global__ __launch_bounds__(RED_THREADS) void k_monitor_partial(KArgs A, const double* __restrict__ U,
                                                                 double p_ref, double ur0, double ur1,
                                                                 double ur2, double* __restrict__ part) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int NF = DIM + 5;
  const long long n = A.E * NN;
  double acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.0;
  double amin = INFINITY, amax = -INFINITY, dp = 0.0, du = 0.0, bad = 0.0;
  const double ur[3] = {ur0, ur1, ur2};
  for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
       i += (long long)gridDim.x * RED_THREADS) {
    const int node = (int)(i % NN);
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int a = (node >> (2 * k)) & 3;
      W *= sel4(a, A.wJ[k][0], A.wJ[k][1], A.wJ[k][2], A.wJ[k][3]);
    }
    double q[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      q[f] = U[f * n + i];
      acc[f] = fma(W, q[f], acc[f]);
    }
    const double al = q[3 + DIM];
    amin = fmin(amin, al);
    amax = fmax(amax, al);
    Prim p;
    closure<DIM>(A, q, p);
    const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
    const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
    const bool nonphys = !(p.rho > 0.0) || !(xi * p.rho > 0.0) || !((1.0 + xi) * p.P + pi > 0.0) ||
                         !isfinite(p.P) || !isfinite(p.c);
    bad += nonphys ? 1.0 : 0.0;
    dp = fmax(dp, fabs(p.P - p_ref));
#pragma unroll
    for (int j = 0; j < DIM; ++j) du = fmax(du, fabs(p.u[j] - ur[j]));
  }
  __shared__ double sh[MON_SLOTS][RED_THREADS / 64];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const double v = wave_sum(acc[f]);
    if ((threadIdx.x & 63) == 0) sh[f][w] = v;
  }
  {
    const double v0 = wave_min(amin), v1 = wave_max(amax), v2 = wave_max(dp), v3 = wave_max(du),
                 v4 = wave_sum(bad);
    if ((threadIdx.x & 63) == 0) {
      sh[NF][w] = v0;
      sh[NF + 1][w] = v1;
      sh[NF + 2][w] = v2;
      sh[NF + 3][w] = v3;
      sh[NF + 4][w] = v4;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + (long long)blockIdx.x * MON_SLOTS;
    for (int f = 0; f < NF; ++f) {
      double v = sh[f][0];
      for (int i = 1; i < RED_THREADS / 64; ++i) v += sh[f][i];
      o[f] = v;
    }
    double v0 = sh[NF][0], v1 = sh[NF + 1][0], v2 = sh[NF + 2][0], v3 = sh[NF + 3][0],
           v4 = sh[NF + 4][0];
    for (int i = 1; i < RED_THREADS / 64; ++i) {
      v0 = fmin(v0, sh[NF][i]);
      v1 = fmax(v1, sh[NF + 1][i]);
      v2 = fmax(v2, sh[NF + 2][i]);
      v3 = fmax(v3, sh[NF + 3][i]);
      v4 += sh[NF + 4][i];
    }
    o[NF] = v0;
    o[NF + 1] = v1;
    o[NF + 2] = v2;
    o[NF + 3] = v3;
    o[NF + 4] = v4;
  }
}

template <int DIM>
__global__ __launch_bounds__(64) void k_monitor_final(const double* __restrict__ part, int nblk,
                                                      dg2p_monitors* mon) {
  constexpr int NF = DIM + 5;
  // one lane per slot, blocks summed in index order (deterministic)
  const int t = threadIdx.x;
  if (t >= NF + 5) return;
  double v = part[t];
  for (int b = 1; b < nblk; ++b) {
    const double x = part[(long long)b * MON_SLOTS + t];
    if (t < NF || t == NF + 4)
      v += x;
    else if (t == NF)
      v = fmin(v, x);
    else
      v = fmax(v, x);
  }
  if (t < NF)
    mon->integral[t] = v;
  else if (t == NF)
    mon->min_alpha = v;
  else if (t == NF + 1)
    mon->max_alpha = v;
  else if (t == NF + 2)
    mon->dev_p = v;
  else if (t == NF + 3)
    mon->dev_u = v;
  else
    mon->nonphys = (long long)v;
}

}  // namespace dg2p
