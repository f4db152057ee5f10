// Kinematic mode: the phase field phi and the level set psi under a
// prescribed velocity u(x, t) = u0(x) s(t) (Results, "Kinematic tests": the
// interface-capturing technique on its own).  The discretisation is that of
// the phi and psi rows of the stage kernel: transport u.grad as a volume
// source plus the hat/tilde face correction, the Allen-Cahn flux
// a = Gamma (eps grad phi - phi (1-phi) n) with n from grad psi, symmetric
// interior penalty for the a-fluxes.  With no sound speed the face speed is
// lambda = max |u.m| over both traces, which makes the hat/tilde correction
// the upwind flux.  Periodic meshes.
//
// State: P[0] = phi, P[1] = psi, each [E][(p+1)^d]; velocity amplitude
// u0[k][E][(p+1)^d]; face ingredients G[2k + side][E][face node] = a.e_k.
// Lane mapping, contractions, XCD-aware workgroup order and the owner-computes
// face evaluation are those of the stage kernel.

#pragma once

#include "dg2p_device.hpp"

namespace dg2p {

struct KinIO {
  const double* Ps;  // stage input
  const double* Gin; // a.e_k of Ps
  const double* u0;  // velocity amplitude
  double s;          // time factor of the stage
  const double* Pn;  // base state of the stage combination (may equal Out)
  double* Acc;       // RK4 accumulator
  double* Out;       // R (MODE 0) or the next state
  double* Gout;      // a.e_k of Out (MODE 1, 2)
  double cdt;        // MODE 1: Out = Pn + cdt R
  double wacc;       // MODE 1: Acc = (first ? 0 : Acc) + wacc R
  int acc_first;
  double dt6;        // MODE 2: Out = Pn + dt6 (Acc + R)
};

template <int DIM>
__device__ __forceinline__ void kin_flux(const KArgs& A, double phi, const double* gphi, const double* gpsi,
                                         double* a) {
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) g2 = fma(gpsi[k], gpsi[k], g2);
  const double inv = rsqrt_nr(g2 + A.delta * A.delta);
  const double pp = phi * (1.0 - phi);
#pragma unroll
  for (int k = 0; k < DIM; ++k) a[k] = A.Gamma * (A.eps * gphi[k] - pp * (gpsi[k] * inv));
}

// a.e_k of a lane's (phi, psi) on the element's own faces -> G.
template <int DIM>
__device__ __forceinline__ void kin_emit(const KArgs& A, double phi, double psi, long long e, bool valid, int node,
                                         const int* ak, const LaneD<DIM>& L, double* G) {
  constexpr int NFN = (1 << (2 * DIM)) / 4;
  double gphi[DIM], gpsi[DIM], a[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    gphi[k] = dk<DIM>(phi, k, L, A);
    gpsi[k] = dk<DIM>(psi, k, L, A);
  }
  kin_flux<DIM>(A, phi, gphi, gpsi, a);
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (ak[k] != 0 && ak[k] != 3) continue;
    const int side = ak[k] == 3;
    G[((long long)(2 * k + side) * A.E + e) * NFN + face_index(node, k)] = a[k];
  }
}

template <int DIM>
__global__ __launch_bounds__(ewg<DIM>()) void k_kin_ingredients(KArgs A, const double* __restrict__ P,
                                                           double* __restrict__ G) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
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
  LaneD<DIM> L;
  lane_coeffs<DIM>(A, ak, L);
  const long long fs = A.E * NN;
  const long long o = e * NN + node;
  kin_emit<DIM>(A, P[o], P[fs + o], e, valid, node, ak, L, G);
}

// MODE 0: Out = R.  MODE 1: Acc = (first ? 0 : Acc) + wacc R, Out = Pn + cdt R,
// and Gout for Out.  MODE 2: Out = Pn + dt6 (Acc + R) and Gout for Out.
template <int DIM, int MODE>
__global__ __launch_bounds__(ewg<DIM>()) void k_kin_stage(KArgs A, KinIO io) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
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
  LaneD<DIM> L;
  lane_coeffs<DIM>(A, ak, L);
  const long long fs = A.E * NN;
  const long long o = e * NN + node;
  const double* __restrict__ Ps = io.Ps;
  const double phi = Ps[o], psi = Ps[fs + o];
  double u[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) u[k] = io.s * io.u0[k * fs + o];
  double gphi[DIM], gpsi[DIM], a[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    gphi[k] = dk<DIM>(phi, k, L, A);
    gpsi[k] = dk<DIM>(psi, k, L, A);
  }
  kin_flux<DIM>(A, phi, gphi, gpsi, a);
  // volume: -u.grad phi + div a, -u.grad psi
  double Rphi = 0.0, Rpsi = 0.0, ua = 0.0, up = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    Rphi += dk<DIM>(a[k], k, L, A);
    ua = fma(u[k], gphi[k], ua);
    up = fma(u[k], gpsi[k], up);
  }
  Rphi -= ua;
  Rpsi = -up;
  // element multi-index
  long long ec[3] = {0, 0, 0};
  elem_coords<DIM>(A, e, ec);
  // faces (periodic neighbours)
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int S = 1 << (2 * k);
    const int akk = ak[k];
    const bool isface = (akk == 0) || (akk == 3);
    double symv = 0.0;
    if (isface) {
      const int side = akk == 3;
      const double sm = side ? 1.0 : -1.0;
      long long c = ec[k] + (side ? 1 : -1);
      if (c < 0) c = A.N[k] - 1;
      if (c >= A.N[k]) c = 0;
      long long estr = 1;
#pragma unroll
      for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
      const long long en = e + (c - ec[k]) * estr;
      const long long oe = en * NN + node + (3 - 2 * akk) * S;
      const double phie = Ps[oe], psie = Ps[fs + oe];
      const double uek = io.s * io.u0[k * fs + oe];
      const double aek = io.Gin[((long long)(2 * k + 1 - side) * A.E + en) * NFN + face_index(node, k)];
      const double umI = sm * u[k], umE = sm * uek;
      const double lam = fmax(fabs(umI), fabs(umE));
      const double amI = sm * a[k], amE = sm * aek;
      const double jump = phi - phie;
      const double ahat = 0.5 * (amI + amE) - A.pen[k] * A.GammaEps * jump;
      const double Lf = A.lift[k];
      Rphi += Lf * (0.5 * (lam - umI) * (phie - phi) + (ahat - amI));
      Rpsi += Lf * (0.5 * (lam - umI) * (psie - psi));
      symv = sm * A.GammaEps * jump;
    }
    // SIPG symmetric term along the normal line through each face node
    const double wlo = kCoef.sp[0][akk] * A.hJ2inv[k];
    const double whi = kCoef.sp[1][akk] * A.hJ2inv[k];
    double lo, hi;
    if (k == 0) {
      lo = line_end<0>(symv, akk, false);
      hi = line_end<0>(symv, akk, true);
    } else if (k == 1) {
      lo = line_end<1>(symv, akk, false);
      hi = line_end<1>(symv, akk, true);
    } else {
      lo = line_end<2>(symv, akk, false);
      hi = line_end<2>(symv, akk, true);
    }
    Rphi = fma(lo, wlo, fma(hi, whi, Rphi));
  }

  if constexpr (MODE == 0) {
    if (valid) {
      io.Out[o] = Rphi;
      io.Out[fs + o] = Rpsi;
    }
  } else {
    double nphi, npsi;
    if constexpr (MODE == 1) {
      if (valid) {
        const double a0 = io.acc_first ? 0.0 : io.Acc[o];
        const double a1 = io.acc_first ? 0.0 : io.Acc[fs + o];
        io.Acc[o] = a0 + io.wacc * Rphi;
        io.Acc[fs + o] = a1 + io.wacc * Rpsi;
      }
      nphi = io.Pn[o] + io.cdt * Rphi;
      npsi = io.Pn[fs + o] + io.cdt * Rpsi;
    } else {
      nphi = io.Pn[o] + io.dt6 * (io.Acc[o] + Rphi);
      npsi = io.Pn[fs + o] + io.dt6 * (io.Acc[fs + o] + Rpsi);
    }
    if (valid) {
      io.Out[o] = nphi;
      io.Out[fs + o] = npsi;
    }
    kin_emit<DIM>(A, nphi, npsi, e, valid, node, ak, L, io.Gout);
  }
}

// Rate records of the kinematic time step: largest sum_k |u0_k| per workgroup
// (the time factor is at most 1); the diffusive part Gamma eps enters through
// the rate rule's nu_max = max(Gamma eps, 0).
template <int DIM>
__global__ __launch_bounds__(ewg<DIM>()) void k_kin_rate(KArgs A, const double* __restrict__ u0,
                                                    double* __restrict__ rec) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
  const long long blk = logical_block(A);
  if (blk < 0) return;
  const int lane = threadIdx.x & 63;
  const long long e0 = (blk * (ewg<DIM>() / 64) + (threadIdx.x >> 6)) * EPW + lane / NN;
  const bool valid = e0 < A.E;
  const long long e = valid ? e0 : A.E - 1;
  const long long fs = A.E * NN;
  const long long o = e * NN + lane % NN;
  double w = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) w += fabs(u0[k * fs + o]);
  block_rate_record<ewg<DIM>()>(valid ? w : 0.0, 0.0, rec, blk);
}

// Per-workgroup sums of W |phi - phi0|, W (phi - phi0), W phi0 (GLL
// quadrature of the L1 error and of the mass-error numerator and denominator).
constexpr int KERR = 4;
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_kin_errors(KArgs A, const double* __restrict__ phi,
                                                      const double* __restrict__ phi0, double* __restrict__ rec) {
  constexpr int NN = 1 << (2 * DIM);
  const long long n = A.E * NN;
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  double v[KERR] = {0.0, 0.0, 0.0, 0.0};
  if (i < n) {
    const int node = (int)(i % NN);
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int a = (node >> (2 * k)) & 3;
      W *= kCoef.w[a] * A.J[k];
    }
    const double d = phi[i] - phi0[i];
    v[0] = W * fabs(d);
    v[1] = W * d;
    v[2] = W * phi0[i];
  }
  __shared__ double sh[BLOCK / 64][KERR];
#pragma unroll
  for (int s = 0; s < KERR; ++s) {
    const double x = wave_sum(v[s]);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][s] = x;
  }
  __syncthreads();
  if (threadIdx.x < KERR) {
    double x = sh[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < BLOCK / 64; ++w) x += sh[w][threadIdx.x];
    rec[(long long)blockIdx.x * KERR + threadIdx.x] = x;
  }
}

// Sum n records of KERR slots in a fixed order (one workgroup): out[s], s < nout.
static __global__ __attribute__((unused)) __launch_bounds__(FIN_THREADS) void k_kin_sum(const double* __restrict__ rec, long long n, int nout,
                                                         double* __restrict__ out) {
  const int s = threadIdx.x % KERR;
  double acc = 0.0;
  for (long long r = threadIdx.x / KERR; r < n; r += FIN_THREADS / KERR) acc += rec[r * KERR + s];
#pragma unroll
  for (int m = KERR; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
  __shared__ double sh[FIN_THREADS / 64][KERR];
  if ((threadIdx.x & 63) < KERR) sh[threadIdx.x >> 6][s] = acc;
  __syncthreads();
  if (threadIdx.x < nout && threadIdx.x < KERR) {
    double x = sh[0][s];
    for (int i = 1; i < FIN_THREADS / 64; ++i) x += sh[i][s];
    out[s] = x;
  }
}

// ---- level-set re-initialisation ----------------------------------------------
// Pseudo-time iteration d psi / d tau = sgn (1 - |grad psi|) + div(nu grad psi)
// from psi0 = phi - 1/2, sgn = tanh(psi0 / (2 eps |grad psi0|)) (the
// re-initialisation of the Section "Discontinuous Galerkin discretisation",
// with the source sign that relaxes |grad psi| towards 1).  The diffusive
// flux nu grad psi uses the symmetric interior penalty discretisation of the
// a-fluxes, with KArgs.GammaEps = nu.  Single field psi [E][(p+1)^d].

struct ReinitIO {
  const double* Ps;  // stage input psi
  const double* Gin; // nu d_k psi of Ps on the element faces
  const double* sgn; // smeared sign
  const double* Pn;  // base of the stage combination (may equal Out)
  double* Acc;
  double* Out;
  double* Gout;
  double cdt, wacc;
  int acc_first;
  double dt6;
};

template <int DIM>
__device__ __forceinline__ void reinit_emit(const KArgs& A, double psi, long long e, bool valid, int node,
                                            const int* ak, const LaneD<DIM>& L, double* G) {
  constexpr int NFN = (1 << (2 * DIM)) / 4;
  double g[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) g[k] = dk<DIM>(psi, k, L, A);
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (ak[k] != 0 && ak[k] != 3) continue;
    const int side = ak[k] == 3;
    G[((long long)(2 * k + side) * A.E + e) * NFN + face_index(node, k)] = A.GammaEps * g[k];
  }
}

// psi0 = phi - 1/2 -> psi, smeared sign -> sgn, face ingredients of psi0 -> G.
template <int DIM>
__global__ __launch_bounds__(ewg<DIM>()) void k_reinit_start(KArgs A, const double* __restrict__ phi, double eps_phase,
                                                        double* __restrict__ psi, double* __restrict__ sgn,
                                                        double* __restrict__ G) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
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
  LaneD<DIM> L;
  lane_coeffs<DIM>(A, ak, L);
  const long long o = e * NN + node;
  const double p0 = phi[o] - 0.5;
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double gk = dk<DIM>(p0, k, L, A);
    g2 = fma(gk, gk, g2);
  }
  const double nrm = sqrt(g2 + A.delta * A.delta);
  if (valid) {
    psi[o] = p0;
    sgn[o] = tanh(p0 / (2.0 * eps_phase * nrm));
  }
  reinit_emit<DIM>(A, p0, e, valid, node, ak, L, G);
}

// MODE 1: Acc = (first ? 0 : Acc) + wacc R, Out = Pn + cdt R (+ Gout);
// MODE 2: Out = Pn + dt6 (Acc + R) (+ Gout).
template <int DIM, int MODE>
__global__ __launch_bounds__(ewg<DIM>()) void k_reinit_stage(KArgs A, ReinitIO io) {
  constexpr int NN = 1 << (2 * DIM);
  constexpr int EPW = 64 / NN;
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
  LaneD<DIM> L;
  lane_coeffs<DIM>(A, ak, L);
  const long long o = e * NN + node;
  const double* __restrict__ Ps = io.Ps;
  const double psi = Ps[o];
  double g[DIM];
  double g2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    g[k] = dk<DIM>(psi, k, L, A);
    g2 = fma(g[k], g[k], g2);
  }
  double R = io.sgn[o] * (1.0 - sqrt(g2));
#pragma unroll
  for (int k = 0; k < DIM; ++k) R += dk<DIM>(A.GammaEps * g[k], k, L, A);
  long long ec[3] = {0, 0, 0};
  elem_coords<DIM>(A, e, ec);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const int S = 1 << (2 * k);
    const int akk = ak[k];
    const bool isface = (akk == 0) || (akk == 3);
    double symv = 0.0;
    if (isface) {
      const int side = akk == 3;
      const double sm = side ? 1.0 : -1.0;
      long long c = ec[k] + (side ? 1 : -1);
      if (c < 0) c = A.N[k] - 1;
      if (c >= A.N[k]) c = 0;
      long long estr = 1;
#pragma unroll
      for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
      const long long en = e + (c - ec[k]) * estr;
      const double psie = Ps[en * NN + node + (3 - 2 * akk) * S];
      const double aek = io.Gin[((long long)(2 * k + 1 - side) * A.E + en) * NFN + face_index(node, k)];
      const double amI = sm * A.GammaEps * g[k], amE = sm * aek;
      const double jump = psi - psie;
      const double ahat = 0.5 * (amI + amE) - A.pen[k] * A.GammaEps * jump;
      R += A.lift[k] * (ahat - amI);
      symv = sm * A.GammaEps * jump;
    }
    const double wlo = kCoef.sp[0][akk] * A.hJ2inv[k];
    const double whi = kCoef.sp[1][akk] * A.hJ2inv[k];
    double lo, hi;
    if (k == 0) {
      lo = line_end<0>(symv, akk, false);
      hi = line_end<0>(symv, akk, true);
    } else if (k == 1) {
      lo = line_end<1>(symv, akk, false);
      hi = line_end<1>(symv, akk, true);
    } else {
      lo = line_end<2>(symv, akk, false);
      hi = line_end<2>(symv, akk, true);
    }
    R = fma(lo, wlo, fma(hi, whi, R));
  }
  double np;
  if constexpr (MODE == 1) {
    if (valid) io.Acc[o] = (io.acc_first ? 0.0 : io.Acc[o]) + io.wacc * R;
    np = io.Pn[o] + io.cdt * R;
  } else {
    np = io.Pn[o] + io.dt6 * (io.Acc[o] + R);
  }
  if (valid) io.Out[o] = np;
  reinit_emit<DIM>(A, np, e, valid, node, ak, L, io.Gout);
}

}  // namespace dg2p
