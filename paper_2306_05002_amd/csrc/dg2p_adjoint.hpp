// Hand-written vector-Jacobian product (reverse mode) of the residual.
//
// Given a cotangent Rb of R(U), computes Ub = (dR/dU)^T Rb and the surface
// tension cotangent <Rb, dR/dsigma>.  Two passes, owner computes in reverse:
//
//   k_vjp_local  every element recomputes its forward quantities and
//                back-propagates its own residual cotangent through the
//                sources, the volume terms (transposed derivative
//                contractions), the SIPG symmetric term and its faces.  What
//                lands on its own nodes is written to T; what lands on the
//                neighbour's trace (N_f values per face node) and on the
//                neighbour's face ingredients (a.e_k, tau.e_k) is written to
//                the element's own slot of the face buffer FB.
//   k_vjp_gather every element adds what its neighbours left for it in FB:
//                trace cotangents directly, ingredient cotangents through its
//                own gradients (transposed contractions again).
//
// No atomics, fixed reduction order: deterministic.  Non-smooth points follow
// the convention d max(a, b) = 1/2, 1/2 at ties and d|x|/dx = 0 at x = 0.
// Boundary faces: the ghost trace is a function of the element's own trace
// and gradients (ghost_fwd, as in the forward face evaluation), so its
// cotangents go back to the element's own values (ghost_rev) instead of into
// the face buffer, and the gather pass skips those faces.  FP64 only.

#pragma once

#include "dg2p_device.hpp"

namespace dg2p {

// transposed rotated coefficients: lane b receives from the lane whose node
// index along the axis is a, and multiplies by D[a][b]
constexpr double CXT(int b, int r) { return GLL.D[(b + r) & 3][b]; }
constexpr double CYT(int b, int r) { return GLL.D[(b - r) & 3][b]; }
constexpr double CZT(int b, int r) { return GLL.D[b ^ r][b]; }

// the same as a table read with the lane's own a_k (see CoefTab)
struct CoefTabT {
  double c[3][4][4];
};
constexpr CoefTabT make_coef_tab_t() {
  CoefTabT t{};
  for (int b = 0; b < 4; ++b)
    for (int r = 0; r < 4; ++r) {
      t.c[0][b][r] = CXT(b, r);
      t.c[1][b][r] = CYT(b, r);
      t.c[2][b][r] = CZT(b, r);
    }
  return t;
}
static __constant__ CoefTabT kCoefT = make_coef_tab_t();

template <int DIM>
__device__ __forceinline__ void lane_coeffs_T(const KArgs& A, const int* ak, LaneD<DIM>& L) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
#pragma unroll
    for (int r = 0; r < 4; ++r) L.c[k][r] = kCoefT.c[k][ak[k]][r];
  }
  // transposed z-operator (1/J_z) D^T on the matrix cores: entry [a_x][a_z] = D[a_z][a_x]
  L.mz = DIM == 3 ? kCoef.d[ak[DIM == 3 ? 2 : 0]][ak[0]] * A.Jinv[2] : 0.0;
}

// Sum of x over the 4 lanes of the lane's line along axis k.
template <int DIM>
__device__ __forceinline__ double line_sum(double x, int k) {
  if (k == 0) return x + qrot<1>(x) + qrot<2>(x) + qrot<3>(x);
  if (DIM > 1 && k == 1) return x + rrot<1>(x) + rrot<2>(x) + rrot<3>(x);
  return x + __shfl_xor(x, 16) + __shfl_xor(x, 32) + __shfl_xor(x, 48);
}

struct PrimBar {
  double rho, u[3], kin, P, c, sE;
};

__device__ __forceinline__ void zero(PrimBar& b) {
  b.rho = b.kin = b.P = b.c = b.sE = 0.0;
  b.u[0] = b.u[1] = b.u[2] = 0.0;
}

// Reverse of closure(): accumulate into qb the cotangent of q given the
// cotangents of (rho, u, kin, P, c, sE).
template <int DIM>
__device__ __forceinline__ void closure_rev(const KArgs& A, const double* q, const Prim& p, const PrimBar& b,
                                            double* qb) {
  const double al = q[3 + DIM];
  const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
  const double pi = al * A.pi1 + (1.0 - al) * A.pi2;
  double Pb = b.P + (A.gh1 - A.gh2) * b.sE;
  double xib = 0.0, pib = 0.0, rhob = b.rho;
  {  // c = sqrt(N / Dn), N = (1 + xi) P + pi, Dn = xi rho
    const double N = (1.0 + xi) * p.P + pi, Dn = xi * p.rho;
    const double Xb = b.c / (2.0 * p.c);
    const double Nb = Xb / Dn;
    const double Dnb = -Xb * (N / Dn) / Dn;
    Pb += (1.0 + xi) * Nb;
    xib += p.P * Nb;
    pib += Nb;
    xib += p.rho * Dnb;
    rhob += xi * Dnb;
  }
  // P = (rho e - pi) / xi
  const double rhoeb = Pb / xi;
  pib -= Pb / xi;
  xib -= Pb * p.P / xi;
  const double alb = (A.xi1 - A.xi2) * xib + (A.pi1 - A.pi2) * pib;
  // rho e = rho E - rho kin
  qb[2 + DIM] += rhoeb;
  rhob -= p.kin * rhoeb;
  const double kinb = b.kin - p.rho * rhoeb;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double ub = b.u[j] + p.u[j] * kinb;
    qb[2 + j] += ub / p.rho;
    rhob -= ub * p.u[j] / p.rho;
  }
  qb[0] += rhob;
  qb[1] += rhob;
  qb[3 + DIM] += alb;
}

template <int DIM>
__device__ __forceinline__ void s_coef_rev(const KArgs& A, int qi, double sb, PrimBar& b) {
  const double dr = A.rho01 - A.rho02;
  if (qi < 2) return;
  if (qi < 2 + DIM) {
    b.u[qi - 2] += dr * sb;
  } else {
    b.kin += dr * sb;
    b.sE += sb;
  }
}

template <int DIM>
__device__ __forceinline__ void conv_flux_rev(const double* q, const Prim& p, int qi, int k, double Fb, double* qb,
                                              PrimBar& b) {
  if (qi < 2 + DIM) {
    qb[qi] += p.u[k] * Fb;
    b.u[k] += q[qi] * Fb;
    if (qi >= 2 && qi - 2 == k) b.P += Fb;
  } else {
    qb[2 + DIM] += p.u[k] * Fb;
    b.P += p.u[k] * Fb;
    b.u[k] += (q[2 + DIM] + p.P) * Fb;
  }
}

// Forward gradient quantities the reverse pass needs.
template <int DIM, bool VISC>
struct GradF {
  double gA[DIM], gP[DIM], nh[DIM], a[DIM], inv;
  double S[VISC ? DIM : 1][VISC ? DIM : 1];
  double mu;
};

template <int DIM, bool VISC>
__device__ __forceinline__ void gradients_fwd(const KArgs& A, const double* q, const Prim& p, const LaneD<DIM>& L,
                                              GradF<DIM, VISC>& g) {
  const double al = q[3 + DIM], ps = q[4 + DIM];
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    g.gA[k] = dk<DIM>(al, k, L, A);
    g.gP[k] = dk<DIM>(ps, k, L, A);
    g2 = fma(g.gP[k], g.gP[k], g2);
  }
  g.inv = 1.0 / sqrt(g2 + A.delta * A.delta);
  const double aa = al * (1.0 - al);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    g.nh[k] = g.gP[k] * g.inv;
    g.a[k] = A.Gamma * (A.eps * g.gA[k] - aa * g.nh[k]);
  }
  if constexpr (VISC) {
    double gU[DIM][DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k) gU[j][k] = dk<DIM>(p.u[j], k, L, A);
    double div = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) div += gU[j][j];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
#pragma unroll
      for (int k = 0; k < DIM; ++k) g.S[j][k] = gU[j][k] + gU[k][j] - (j == k ? (2.0 / 3.0) * div : 0.0);
    g.mu = A.mu1 * al + A.mu2 * (1.0 - al);
  } else {
    g.mu = 0.0;
  }
}

// Reverse of the gradient quantities: given cotangents of a, n, grad alpha,
// grad psi, S and mu (per node), accumulate into qb (alpha, psi) and ub (u).
template <int DIM, bool VISC>
__device__ __forceinline__ void gradients_rev(const KArgs& A, const double* q, const GradF<DIM, VISC>& g,
                                              const LaneD<DIM>& LT, double* ab, double* nhb, double* gAb,
                                              double* gPb, double (*Sb)[VISC ? DIM : 1], double mub, double* qb,
                                              double* ub) {
  const double al = q[3 + DIM];
  const double aa = al * (1.0 - al);
  double aab = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    gAb[k] += A.Gamma * A.eps * ab[k];
    aab -= A.Gamma * g.nh[k] * ab[k];
    nhb[k] -= A.Gamma * aa * ab[k];
  }
  qb[3 + DIM] += (1.0 - 2.0 * al) * aab;
  double nn = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) nn += g.nh[k] * nhb[k];
#pragma unroll
  for (int k = 0; k < DIM; ++k) gPb[k] += g.inv * (nhb[k] - g.nh[k] * nn);
  double alb = 0.0, psb = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    alb += dk<DIM>(gAb[k], k, LT, A);
    psb += dk<DIM>(gPb[k], k, LT, A);
  }
  qb[3 + DIM] += alb;
  qb[4 + DIM] += psb;
  if constexpr (VISC) {
    qb[3 + DIM] += (A.mu1 - A.mu2) * mub;
    double tr = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) tr += Sb[j][j];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double gUb = Sb[j][k] + Sb[k][j] - (j == k ? (2.0 / 3.0) * tr : 0.0);
        acc += dk<DIM>(gUb, k, LT, A);
      }
      ub[j] += acc;
    }
  }
}

struct VjpIO {
  const double* U;     // state
  const double* Gin;   // face ingredients of U
  const double* Rb;    // cotangent of R
  double* T;           // own-node cotangent (local pass)
  double* FB;          // face buffer [slot][comp][E][face node], comp < N_f: trace, then ingredients
  double* rec;         // per-workgroup surface-tension cotangent (local pass)
  double* Out;         // gather pass output
  int accumulate;      // gather: Out += result (else Out = result)
};

template <int WT>
__device__ __forceinline__ void block_sum(double v, double* rec, long long blk) {
  __shared__ double sh[WT / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = sh[0];
#pragma unroll
    for (int i = 1; i < WT / 64; ++i) x += sh[i];
    rec[blk] = x;
  }
}

// Ghost trace of a boundary face (axis kd, side, boundary kind) from the
// element's own trace q, pr and gradient quantities g: the neighbour state qe,
// its a.e_kd (aek) and viscous traction (tek), built as in face_flux.
template <int DIM, bool VISC>
__device__ __forceinline__ void ghost_fwd(const KArgs& A, int kd, int side, int kind, const double* q,
                                          const Prim& pr, const GradF<DIM, VISC>& g, double* qe, double& aek,
                                          double* tek) {
  constexpr int NF = DIM + 5;
  const double sm = side ? 1.0 : -1.0;
#pragma unroll
  for (int f = 0; f < NF; ++f) qe[f] = q[f];
  aek = g.a[kd];
  if constexpr (VISC) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) tek[j] = g.mu * g.S[j][kd];
  }
  if (kind == DG2P_BC_SLIP_WALL || kind == DG2P_BC_NO_SLIP) {
    const bool slip = kind == DG2P_BC_SLIP_WALL;
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      if (!slip || j == kd) qe[2 + j] = -q[2 + j];
    aek = -g.a[kd];
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        if (slip && j != kd) tek[j] = -tek[j];
    }
  } else if (kind == DG2P_BC_RIEMANN) {
    const double al = q[3 + DIM];
    const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
    const double pim = al * A.pi1 + (1.0 - al) * A.pi2;
    const double Pb = A.bcs[kd][side][0];
    const double un = sm * pr.u[kd];
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
  } else if (kind == DG2P_BC_DIRICHLET) {
#pragma unroll
    for (int f = 0; f < 4 + DIM; ++f) qe[f] = A.bcs[kd][side][f];
    const double ag = qe[3 + DIM];
    aek = A.Gamma * (A.eps * g.gA[kd] - (ag * (1.0 - ag)) * g.nh[kd]);
    if constexpr (VISC) {
      const double mug = A.mu1 * ag + A.mu2 * (1.0 - ag);
#pragma unroll
      for (int j = 0; j < DIM; ++j) tek[j] = mug * g.S[j][kd];
    }
  }
}

// Reverse of ghost_fwd: the cotangents qeb, aekb, tekb of the ghost trace
// added to the element's own trace (qb, and pb for the primitives the
// Riemann ghost is built from) and gradient quantities (ab, gAb, nhb, Sb, mub).
template <int DIM, bool VISC>
__device__ __forceinline__ void ghost_rev(const KArgs& A, int kd, int side, int kind, const double* q,
                                          const Prim& pr, const GradF<DIM, VISC>& g, const double* qeb,
                                          double aekb, const double* tekb, double* qb, PrimBar& pb, double* ab,
                                          double* gAb, double* nhb, double (*Sb)[VISC ? DIM : 1], double& mub) {
  constexpr int NF = DIM + 5;
  const double sm = side ? 1.0 : -1.0;
  if (kind == DG2P_BC_DIRICHLET) {
    // prescribed (q1, q2, rho u, rho E, alpha); psi and the gradients interior
    qb[4 + DIM] += qeb[4 + DIM];
    const double ag = A.bcs[kd][side][3 + DIM];
    gAb[kd] += A.Gamma * A.eps * aekb;
    nhb[kd] -= A.Gamma * (ag * (1.0 - ag)) * aekb;
    if constexpr (VISC) {
      const double mug = A.mu1 * ag + A.mu2 * (1.0 - ag);
#pragma unroll
      for (int j = 0; j < DIM; ++j) Sb[j][kd] += mug * tekb[j];
    }
    return;
  }
  const bool mirror = kind == DG2P_BC_SLIP_WALL || kind == DG2P_BC_NO_SLIP;
  const bool slip = kind == DG2P_BC_SLIP_WALL;
  // fields copied from the interior (all but the momentum and energy of a
  // Riemann ghost; momentum components with their mirror sign)
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const bool mom = f >= 2 && f < 2 + DIM;
    if (kind == DG2P_BC_RIEMANN && (mom || f == 2 + DIM)) continue;
    double sgn = 1.0;
    if (mirror && mom && (!slip || f - 2 == kd)) sgn = -1.0;
    qb[f] += sgn * qeb[f];
  }
  ab[kd] += mirror ? -aekb : aekb;
  if constexpr (VISC) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double ts = (slip && j != kd) ? -1.0 : 1.0;
      mub += ts * g.S[j][kd] * tekb[j];
      Sb[j][kd] += ts * g.mu * tekb[j];
    }
  }
  if (kind == DG2P_BC_RIEMANN) {
    // recompute the forward values
    const double al = q[3 + DIM];
    const double xi = al * A.xi1 + (1.0 - al) * A.xi2;
    const double pim = al * A.pi1 + (1.0 - al) * A.pi2;
    const double Pb = A.bcs[kd][side][0];
    const double un = sm * pr.u[kd];
    const double N = (1.0 + xi) * Pb + pim, Dn = xi * pr.rho;
    const double cfar = sqrt(N / Dn);
    const double jout = un + 2.0 * xi * pr.c;
    const double jin = -2.0 * xi * cfar;
    const double unb = 0.5 * (jout + jin);
    const double cb = (jout - jin) / (4.0 * xi);
    const double Pg = (xi * pr.rho * cb * cb - pim) / (1.0 + xi);
    double ug[DIM], k2 = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      ug[j] = pr.u[j] + (j == kd ? sm * (unb - un) : 0.0);
      k2 += ug[j] * ug[j];
    }
    // reverse: qe[2 + j] = rho ug_j, qe[2 + DIM] = xi Pg + pim + rho k2 / 2
    const double Eb = qeb[2 + DIM];
    double rhob = 0.5 * k2 * Eb, xib = Pg * Eb, pimb = Eb;
    const double Pgb = xi * Eb;
    double unbb = 0.0, unb_ = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double ugb = pr.rho * qeb[2 + j] + pr.rho * ug[j] * Eb;
      rhob += ug[j] * qeb[2 + j];
      pb.u[j] += ugb;
      if (j == kd) {
        unbb += sm * ugb;
        unb_ -= sm * ugb;
      }
    }
    // Pg = (xi rho cb^2 - pim) / (1 + xi)
    xib += Pgb * (pr.rho * cb * cb + pim) / ((1.0 + xi) * (1.0 + xi));
    rhob += Pgb * xi * cb * cb / (1.0 + xi);
    const double cbb = Pgb * 2.0 * xi * pr.rho * cb / (1.0 + xi);
    pimb -= Pgb / (1.0 + xi);
    // cb = (jout - jin) / (4 xi), unb = (jout + jin) / 2
    double joutb = cbb / (4.0 * xi) + 0.5 * unbb;
    double jinb = -cbb / (4.0 * xi) + 0.5 * unbb;
    xib -= cbb * cb / xi;
    // jin = -2 xi cfar, jout = un + 2 xi c
    xib -= 2.0 * cfar * jinb;
    const double cfarb = -2.0 * xi * jinb;
    unb_ += joutb;
    xib += 2.0 * pr.c * joutb;
    pb.c += 2.0 * xi * joutb;
    // cfar = sqrt(N / Dn)
    const double Xb = cfarb / (2.0 * cfar);
    const double Nb = Xb / Dn;
    const double Dnb = -Xb * N / (Dn * Dn);
    xib += Pb * Nb + pr.rho * Dnb;
    pimb += Nb;
    rhob += xi * Dnb;
    // un = sm u_kd
    pb.u[kd] += sm * unb_;
    pb.rho += rhob;
    qb[3 + DIM] += (A.xi1 - A.xi2) * xib + (A.pi1 - A.pi2) * pimb;
  }
}

// WALLS: the mesh has non-periodic sides (the ghost code is compiled in only
// then, so that the periodic kernels keep their registers).
template <int DIM, bool VISC, bool CSF, bool WALLS>
__global__ __launch_bounds__(ewg<DIM>()) void k_vjp_local(KArgs A, VjpIO io) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  constexpr int NC = DIM + 3;
  constexpr int C = VISC ? 1 + DIM : 1;
  constexpr int CF = NF + C;
  constexpr int NFN = NN / 4;
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
  LaneD<DIM> L, LT;
  lane_coeffs<DIM>(A, ak, L);
  lane_coeffs_T<DIM>(A, ak, LT);
  const long long fs = A.E * NN;
  const long long o = e * NN + node;

  double q[NF], rb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    q[f] = io.U[f * fs + o];
    rb[f] = valid ? io.Rb[f * fs + o] : 0.0;
  }
  Prim pr;
  closure<DIM>(A, q, pr);
  GradF<DIM, VISC> g;
  gradients_fwd<DIM, VISC>(A, q, pr, L, g);

  double qb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) qb[f] = 0.0;
  PrimBar pb;
  zero(pb);
  double ab[DIM], nhb[DIM], gAb[DIM], gPb[DIM];
  double Sb[VISC ? DIM : 1][VISC ? DIM : 1];
  double mub = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) ab[k] = nhb[k] = gAb[k] = gPb[k] = 0.0;
#pragma unroll
  for (int j = 0; j < (VISC ? DIM : 1); ++j)
#pragma unroll
    for (int k = 0; k < (VISC ? DIM : 1); ++k) Sb[j][k] = 0.0;

  // ---- faces and SIPG symmetric term ----
  long long ec[3] = {0, 0, 0};
  elem_coords<DIM>(A, e, ec);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int S = 1 << (2 * k);
    const int akk = ak[k];
    const bool isface = (akk == 0) || (akk == 3);
    // cotangent of the face values spread by the symmetric term
    const double wlo = kCoef.sp[0][akk] * A.hJ2inv[k];
    const double whi = kCoef.sp[1][akk] * A.hJ2inv[k];
    double symb[NC + 1];
#pragma unroll
    for (int i = 0; i <= NC; ++i) {
      const int f = (i < NC) ? i : 3 + DIM;
      const double slo = line_sum<DIM>(rb[f] * wlo, k);
      const double shi = line_sum<DIM>(rb[f] * whi, k);
      symb[i] = akk == 0 ? slo : (akk == 3 ? shi : 0.0);
    }
    if (isface) {
      const int side = akk == 3;
      const double sm = side ? 1.0 : -1.0;
      long long c = ec[k] + (side ? 1 : -1);
      bool bnd = false;
      if (c < 0 || c >= A.N[k]) {
        if (!WALLS || bc_kind(A, k, side) == DG2P_BC_PERIODIC) {
          c = (c < 0) ? A.N[k] - 1 : 0;
        } else {
          bnd = true;  // ghost: the loads below read the element itself (in bounds, replaced)
          c = ec[k];
        }
      }
      long long estr = 1;
#pragma unroll
      for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
      const long long en = e + (c - ec[k]) * estr;
      const int nodee = node + (3 - 2 * akk) * S;
      const int fn = face_index(node, k);
      double qe[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) qe[f] = io.U[(f * A.E + en) * NN + nodee];
      double gv[2 * GLay<DIM, VISC>::P];
      g_read<DIM, VISC>(A, io.Gin, 2 * k + 1 - side, en, fn, gv);
      const double aek = gv[0];
      double tek[DIM];
      if constexpr (VISC) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) tek[j] = gv[1 + j];
      }
      const int kind = bnd ? bc_kind(A, k, side) : DG2P_BC_PERIODIC;
      double aek_ = aek;
      if constexpr (WALLS) {
        if (bnd) ghost_fwd<DIM, VISC>(A, k, side, kind, q, pr, g, qe, aek_, tek);
      }
      Prim pe;
      closure<DIM>(A, qe, pe);
      const double umI = sm * pr.u[k], umE = sm * pe.u[k];
      const double lA = fabs(umI) + pr.c, lB = fabs(umE) + pe.c;
      const double lam = fmax(lA, lB);
      const double amI = sm * g.a[k], amE = sm * aek_;
      const double alI = q[3 + DIM], alE = qe[3 + DIM];
      const double jump = alI - alE;
      const double ahat = 0.5 * (amI + amE) - A.pen[k] * A.GammaEps * jump;
      const double Lf = A.lift[k];
      double mue = 0.0, etav = 0.0;
      if constexpr (VISC) {
        mue = A.mu1 * alE + A.mu2 * (1.0 - alE);
        etav = A.pen[k] * (0.5 * (g.mu + mue));
      }
      // reverse
      double qeb[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) qeb[f] = 0.0;
      PrimBar pbe;
      zero(pbe);
      double aekb = 0.0, tekb[DIM];
#pragma unroll
      for (int j = 0; j < DIM; ++j) tekb[j] = 0.0;
      double lamb = 0.0, ahatb = 0.0, jumpb = 0.0, umIb = 0.0, amIb = 0.0, amEb = 0.0, etavb = 0.0;
#pragma unroll
      for (int qi = 0; qi < NC; ++qi) {
        const double FmI = sm * conv_flux<DIM>(q, pr, qi, k);
        const double FmE = sm * conv_flux<DIM>(qe, pe, qi, k);
        (void)FmI;
        (void)FmE;
        const double sI = s_coef<DIM>(A, pr, qi), sE = s_coef<DIM>(A, pe, qi);
        const double sbar = 0.5 * (sI + sE);
        const double tb = Lf * rb[qi];
        double FmIb = tb, Fhatb = -tb;
        double sbarb = tb * ahat + symb[qi] * sm * A.GammaEps * jump;
        ahatb += tb * sbar;
        double sIb = -tb * amI;
        amIb -= tb * sI;
        jumpb += symb[qi] * sm * sbar * A.GammaEps;
        if constexpr (VISC) {
          if (qi >= 2) {
            const double Vhatb = tb;
            const double VmIb = -tb + 0.5 * Vhatb, VmEb = 0.5 * Vhatb, penb = -Vhatb;
            if (qi < 2 + DIM) {
              const int j = qi - 2;
              mub += sm * g.S[j][k] * VmIb;
              Sb[j][k] += sm * g.mu * VmIb;
              tekb[j] += sm * VmEb;
              etavb += (pr.u[j] - pe.u[j]) * penb;
              pb.u[j] += etav * penb;
              pbe.u[j] -= etav * penb;
            } else {
              double du = 0.0;
#pragma unroll
              for (int j = 0; j < DIM; ++j) {
                mub += sm * g.S[j][k] * pr.u[j] * VmIb;
                Sb[j][k] += sm * g.mu * pr.u[j] * VmIb;
                pb.u[j] += sm * g.mu * g.S[j][k] * VmIb;
                tekb[j] += sm * pe.u[j] * VmEb;
                pbe.u[j] += sm * tek[j] * VmEb;
                du += (pr.u[j] - pe.u[j]) * (0.5 * (pr.u[j] + pe.u[j]));
                pb.u[j] += etav * penb * pr.u[j];
                pbe.u[j] -= etav * penb * pe.u[j];
              }
              etavb += du * penb;
            }
          }
        }
        // Fhat = 1/2 (FmI + FmE) - 1/2 lam (qe - q)
        FmIb += 0.5 * Fhatb;
        const double FmEb = 0.5 * Fhatb;
        lamb -= 0.5 * (qe[qi] - q[qi]) * Fhatb;
        qeb[qi] -= 0.5 * lam * Fhatb;
        qb[qi] += 0.5 * lam * Fhatb;
        sIb += 0.5 * sbarb;
        const double sEb = 0.5 * sbarb;
        s_coef_rev<DIM>(A, qi, sIb, pb);
        s_coef_rev<DIM>(A, qi, sEb, pbe);
        conv_flux_rev<DIM>(q, pr, qi, k, sm * FmIb, qb, pb);
        conv_flux_rev<DIM>(qe, pe, qi, k, sm * FmEb, qeb, pbe);
      }
      {  // alpha: L (KA + ahat - amI), KA = 1/2 (lam - umI)(alE - alI)
        const double tab = Lf * rb[3 + DIM];
        ahatb += tab;
        amIb -= tab;
        lamb += 0.5 * (alE - alI) * tab;
        umIb -= 0.5 * (alE - alI) * tab;
        qeb[3 + DIM] += 0.5 * (lam - umI) * tab;
        qb[3 + DIM] -= 0.5 * (lam - umI) * tab;
        jumpb += symb[NC] * sm * A.GammaEps;
      }
      {  // psi: L 1/2 (lam - umI)(psE - psI)
        const double tpb = Lf * rb[4 + DIM];
        const double dps = qe[4 + DIM] - q[4 + DIM];
        lamb += 0.5 * dps * tpb;
        umIb -= 0.5 * dps * tpb;
        qeb[4 + DIM] += 0.5 * (lam - umI) * tpb;
        qb[4 + DIM] -= 0.5 * (lam - umI) * tpb;
      }
      amIb += 0.5 * ahatb;
      amEb += 0.5 * ahatb;
      jumpb -= A.pen[k] * A.GammaEps * ahatb;
      qb[3 + DIM] += jumpb;
      qeb[3 + DIM] -= jumpb;
      ab[k] += sm * amIb;
      aekb += sm * amEb;
      if constexpr (VISC) {
        mub += 0.5 * A.pen[k] * etavb;
        qeb[3 + DIM] += (A.mu1 - A.mu2) * 0.5 * A.pen[k] * etavb;
      }
      const double lAb = lA > lB ? lamb : (lB > lA ? 0.0 : 0.5 * lamb);
      const double lBb = lB > lA ? lamb : (lA > lB ? 0.0 : 0.5 * lamb);
      umIb += (umI > 0.0 ? 1.0 : (umI < 0.0 ? -1.0 : 0.0)) * lAb;
      pb.c += lAb;
      const double umEb = (umE > 0.0 ? 1.0 : (umE < 0.0 ? -1.0 : 0.0)) * lBb;
      pbe.c += lBb;
      pb.u[k] += sm * umIb;
      pbe.u[k] += sm * umEb;
      closure_rev<DIM>(A, qe, pe, pbe, qeb);
      if (WALLS && bnd) {
        ghost_rev<DIM, VISC>(A, k, side, kind, q, pr, g, qeb, aekb, tekb, qb, pb, ab, gAb, nhb, Sb, mub);
      } else if (valid) {
        const long long fb = (long long)((2 * k + side) * CF) * A.E;
#pragma unroll
        for (int f = 0; f < NF; ++f) io.FB[(fb + (long long)f * A.E + e) * NFN + fn] = qeb[f];
        io.FB[(fb + (long long)NF * A.E + e) * NFN + fn] = aekb;
        if constexpr (VISC) {
#pragma unroll
          for (int j = 0; j < DIM; ++j) io.FB[(fb + (long long)(NF + 1 + j) * A.E + e) * NFN + fn] = tekb[j];
        }
      }
    }
  }

  // ---- volume terms: R_q += sum_k (1/J_k) D_k (-F_q + s_q a + V_q)_k ----
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) {
    const double sq = s_coef<DIM>(A, pr, qi);
    double sqb = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double fb = dk<DIM>(rb[qi], k, LT, A);  // transposed contraction
      conv_flux_rev<DIM>(q, pr, qi, k, -fb, qb, pb);
      sqb += g.a[k] * fb;
      ab[k] += sq * fb;
      if constexpr (VISC) {
        if (qi >= 2 && qi < 2 + DIM) {
          mub += g.S[qi - 2][k] * fb;
          Sb[qi - 2][k] += g.mu * fb;
        } else if (qi == 2 + DIM) {
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            mub += g.S[j][k] * pr.u[j] * fb;
            Sb[j][k] += g.mu * pr.u[j] * fb;
            pb.u[j] += g.mu * g.S[j][k] * fb;
          }
        }
      }
    }
    s_coef_rev<DIM>(A, qi, sqb, pb);
  }
  // alpha: -u . grad alpha + div a ; psi: -u . grad psi
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    ab[k] += dk<DIM>(rb[3 + DIM], k, LT, A);
    pb.u[k] -= g.gA[k] * rb[3 + DIM] + g.gP[k] * rb[4 + DIM];
    gAb[k] -= pr.u[k] * rb[3 + DIM];
    gPb[k] -= pr.u[k] * rb[4 + DIM];
  }
  // ---- sources ----
  double sigb = 0.0;
  if (A.has_grav) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      pb.rho += A.grav[j] * rb[2 + j] + A.grav[j] * pr.u[j] * rb[2 + DIM];
      pb.u[j] += pr.rho * A.grav[j] * rb[2 + DIM];
    }
  }
  if constexpr (CSF) {
    double div = 0.0, ga2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      div += dk<DIM>(g.nh[k], k, L, A);
      ga2 = fma(g.gA[k], g.gA[k], ga2);
    }
    const double kappa = -div;
    const double rr = sqrt(ga2 + A.delta * A.delta);
    const double dG = rr - A.delta;
    const double csf = A.sigma * kappa * dG;
    double csfb = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      csfb += g.nh[j] * rb[2 + j] + pr.u[j] * g.nh[j] * rb[2 + DIM];
      nhb[j] += csf * rb[2 + j] + csf * pr.u[j] * rb[2 + DIM];
      pb.u[j] += csf * g.nh[j] * rb[2 + DIM];
    }
    const double kappab = A.sigma * dG * csfb;
    const double dGb = A.sigma * kappa * csfb;
    sigb = valid ? kappa * dG * csfb : 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      gAb[k] += dGb * g.gA[k] / rr;
      nhb[k] -= dk<DIM>(kappab, k, LT, A);
    }
  }
  // ---- gradients and closure ----
  double ub[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) ub[j] = 0.0;
  gradients_rev<DIM, VISC>(A, q, g, LT, ab, nhb, gAb, gPb, Sb, mub, qb, ub);
#pragma unroll
  for (int j = 0; j < DIM; ++j) pb.u[j] += ub[j];
  closure_rev<DIM>(A, q, pr, pb, qb);
  if (valid) {
#pragma unroll
    for (int f = 0; f < NF; ++f) io.T[f * fs + o] = qb[f];
  }
  if constexpr (CSF) block_sum<ewg<DIM>()>(sigb, io.rec, blk);
}

template <int DIM, bool VISC, bool WALLS>
__global__ __launch_bounds__(ewg<DIM>()) void k_vjp_gather(KArgs A, VjpIO io) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  constexpr int NF = DIM + 5;
  constexpr int C = VISC ? 1 + DIM : 1;
  constexpr int CF = NF + C;
  constexpr int NFN = NN / 4;
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
  LaneD<DIM> L, LT;
  lane_coeffs<DIM>(A, ak, L);
  lane_coeffs_T<DIM>(A, ak, LT);
  const long long fs = A.E * NN;
  const long long o = e * NN + node;
  double q[NF], qb[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    q[f] = io.U[f * fs + o];
    qb[f] = io.T[f * fs + o];
  }
  Prim pr;
  closure<DIM>(A, q, pr);
  GradF<DIM, VISC> g;
  gradients_fwd<DIM, VISC>(A, q, pr, L, g);
  double ab[DIM], nhb[DIM], gAb[DIM], gPb[DIM];
  double Sb[VISC ? DIM : 1][VISC ? DIM : 1];
  double mub = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) ab[k] = nhb[k] = gAb[k] = gPb[k] = 0.0;
#pragma unroll
  for (int j = 0; j < (VISC ? DIM : 1); ++j)
#pragma unroll
    for (int k = 0; k < (VISC ? DIM : 1); ++k) Sb[j][k] = 0.0;
  long long ec[3] = {0, 0, 0};
  elem_coords<DIM>(A, e, ec);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int akk = ak[k];
    if (akk != 0 && akk != 3) continue;
    const int side = akk == 3;
    long long c = ec[k] + (side ? 1 : -1);
    if (c < 0 || c >= A.N[k]) {
      // a boundary face has no neighbour: its ghost was reversed locally
      if (WALLS && bc_kind(A, k, side) != DG2P_BC_PERIODIC) continue;
      c = (c < 0) ? A.N[k] - 1 : 0;
    }
    long long estr = 1;
#pragma unroll
    for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
    const long long en = e + (c - ec[k]) * estr;
    const int fn = face_index(node, k);
    // the neighbour's slot facing this element
    const long long fb = (long long)((2 * k + 1 - side) * CF) * A.E;
#pragma unroll
    for (int f = 0; f < NF; ++f) qb[f] += io.FB[(fb + (long long)f * A.E + en) * NFN + fn];
    ab[k] += io.FB[(fb + (long long)NF * A.E + en) * NFN + fn];
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const double tb = io.FB[(fb + (long long)(NF + 1 + j) * A.E + en) * NFN + fn];
        mub += g.S[j][k] * tb;
        Sb[j][k] += g.mu * tb;
      }
    }
  }
  double ub[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) ub[j] = 0.0;
  gradients_rev<DIM, VISC>(A, q, g, LT, ab, nhb, gAb, gPb, Sb, mub, qb, ub);
  PrimBar pb;
  zero(pb);
#pragma unroll
  for (int j = 0; j < DIM; ++j) pb.u[j] = ub[j];
  closure_rev<DIM>(A, q, pr, pb, qb);
  if (!valid) return;
#pragma unroll
  for (int f = 0; f < NF; ++f) io.Out[f * fs + o] = (io.accumulate ? io.Out[f * fs + o] : 0.0) + qb[f];
}

// Stage combination of the RK-step reverse pass (one thread per value):
// Ub += an X;  Xo = ax X (if Xo);  Rb = ar dt X.
static __global__ __attribute__((unused)) void k_vjp_combine(long long n, const double* X, const double* dt, double an, int init, double* Ub,
                              double ax, double* Xo, double ar, double* Rb) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = X[i];
  Ub[i] = init ? an * x : Ub[i] + an * x;
  if (Xo) Xo[i] = ax * x;
  Rb[i] = ar * (*dt) * x;
}

// Fixed-order sum of n per-workgroup values added to *out.
static __global__ __attribute__((unused)) __launch_bounds__(BLOCK) void k_sum_add(const double* __restrict__ v, long long n, double* out) {
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += BLOCK) acc += v[i];
  __shared__ double sh[BLOCK / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = sh[0];
    for (int i = 1; i < BLOCK / 64; ++i) x += sh[i];
    *out += x;
  }
}

}  // namespace dg2p
