// Kinematic mode at polynomial degree p = 1 (the first-order rows of the
// paper's Rider-Kothe study, Results, "Kinematic tests").  Same operator as
// dg2p_kinematic.hpp (transport u.grad as a volume source plus the upwind
// hat/tilde face correction for phi and psi, the Allen-Cahn flux
// a = Gamma (eps grad phi - phi (1 - phi) n), n = grad psi / |grad psi|,
// symmetric interior penalty for a), on two GLL nodes per axis: the nodes
// are the element's corners (xi = -1, 1), the weights are 1, 1, and
// D[a][b] = l_b'(xi_a) = (-1/2, 1/2) for both a, so a derivative along k is
// (f_high - f_low) / h_k at either node of the line.
//
// One thread per element: the element has 2^d nodes, node j = sum_k a_k 2^k.
// Each face's neighbour interface flux a.e_k at the shared nodes comes from
// the neighbour's own nodes (loaded whole and differentiated here; no
// face-ingredient buffer).  These runs are small and launch-bound, so the
// kernels favour plain code over lane mappings.

#pragma once

#include "dg2p_device.hpp"
#include "dg2p_kinematic.hpp"

namespace dg2p {

template <int DIM>
struct P1Elem {
  static constexpr int NN = 1 << DIM;
  double phi[NN], psi[NN];
  double gphi[DIM][NN], gpsi[DIM][NN], a[DIM][NN];
};

// Nodal data and element-local gradients / interface flux of element e.
template <int DIM>
__device__ __forceinline__ void p1_elem(const KArgs& A, const double* __restrict__ P, long long e, P1Elem<DIM>& X) {
  constexpr int NN = 1 << DIM;
  const long long fs = A.E * NN;
#pragma unroll
  for (int j = 0; j < NN; ++j) {
    X.phi[j] = P[e * NN + j];
    X.psi[j] = P[fs + e * NN + j];
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double c = 0.5 * A.Jinv[k];  // (f_high - f_low) / (2 J_k)
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      const int lo = j & ~(1 << k), hi = j | (1 << k);
      X.gphi[k][j] = c * (X.phi[hi] - X.phi[lo]);
      X.gpsi[k][j] = c * (X.psi[hi] - X.psi[lo]);
    }
  }
#pragma unroll
  for (int j = 0; j < NN; ++j) {
    double gp[DIM], gs[DIM], av[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      gp[k] = X.gphi[k][j];
      gs[k] = X.gpsi[k][j];
    }
    kin_flux<DIM>(A, X.phi[j], gp, gs, av);
#pragma unroll
    for (int k = 0; k < DIM; ++k) X.a[k][j] = av[k];
  }
}

// Residual of the element and the stage combination of dg2p_kin_rk4 (MODE as
// in k_kin_stage: 0 R, 1 next stage state and accumulator, 2 final update).
template <int DIM, int MODE>
__global__ __launch_bounds__(BLOCK) void k_kin1_stage(KArgs A, KinIO io) {
  constexpr int NN = 1 << DIM;
  const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= A.E) return;
  const long long fs = A.E * NN;
  P1Elem<DIM> X;
  p1_elem<DIM>(A, io.Ps, e, X);
  double u[DIM][NN];
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int j = 0; j < NN; ++j) u[k][j] = io.s * io.u0[k * fs + e * NN + j];
  double Rphi[NN], Rpsi[NN];
  // volume: -u.grad phi + div a, -u.grad psi
#pragma unroll
  for (int j = 0; j < NN; ++j) {
    double rp = 0.0, rs = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int lo = j & ~(1 << k), hi = j | (1 << k);
      rp += 0.5 * A.Jinv[k] * (X.a[k][hi] - X.a[k][lo]) - u[k][j] * X.gphi[k][j];
      rs -= u[k][j] * X.gpsi[k][j];
    }
    Rphi[j] = rp;
    Rpsi[j] = rs;
  }
  // faces
  long long ec[3] = {0, 0, 0};
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
    long long estr = 1;
#pragma unroll
    for (int kk = 0; kk < k; ++kk) estr *= A.N[kk];
    const double L = A.lift[k];
    const double eta = A.pen[k] * A.GammaEps;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const double sm = side ? 1.0 : -1.0;
      long long c = ec[k] + (side ? 1 : -1);
      c = c < 0 ? A.N[k] - 1 : (c >= A.N[k] ? 0 : c);  // periodic
      const long long en = e + (c - ec[k]) * estr;
      P1Elem<DIM> Y;
      p1_elem<DIM>(A, io.Ps, en, Y);
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        if (((j >> k) & 1) != side) continue;
        const int jn = j ^ (1 << k);  // the neighbour's node on the shared face
        const double umI = sm * u[k][j];
        const double umE = sm * io.s * io.u0[k * fs + en * NN + jn];
        const double lam = fmax(fabs(umI), fabs(umE));
        const double amI = sm * X.a[k][j], amE = sm * Y.a[k][jn];
        const double jump = X.phi[j] - Y.phi[jn];
        const double ahat = 0.5 * (amI + amE) - eta * jump;
        Rphi[j] += L * (0.5 * (lam - umI) * (Y.phi[jn] - X.phi[j]) + (ahat - amI));
        Rpsi[j] += L * (0.5 * (lam - umI) * (Y.psi[jn] - X.psi[j]));
        // symmetric term along the normal line: D[side][a] / (2 w_a J_k^2),
        // D[.][0] = -1/2, D[.][1] = 1/2, w = 1
        const double sym = sm * A.GammaEps * jump * A.hJ2inv[k];
        Rphi[j & ~(1 << k)] -= 0.5 * sym;
        Rphi[j | (1 << k)] += 0.5 * sym;
      }
    }
  }
  const long long o = e * NN;
  if constexpr (MODE == 0) {
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      io.Out[o + j] = Rphi[j];
      io.Out[fs + o + j] = Rpsi[j];
    }
  } else if constexpr (MODE == 1) {
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      const double a0 = io.acc_first ? 0.0 : io.Acc[o + j];
      const double a1 = io.acc_first ? 0.0 : io.Acc[fs + o + j];
      io.Acc[o + j] = a0 + io.wacc * Rphi[j];
      io.Acc[fs + o + j] = a1 + io.wacc * Rpsi[j];
      io.Out[o + j] = io.Pn[o + j] + io.cdt * Rphi[j];
      io.Out[fs + o + j] = io.Pn[fs + o + j] + io.cdt * Rpsi[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < NN; ++j) {
      io.Out[o + j] = io.Pn[o + j] + io.dt6 * (io.Acc[o + j] + Rphi[j]);
      io.Out[fs + o + j] = io.Pn[fs + o + j] + io.dt6 * (io.Acc[fs + o + j] + Rpsi[j]);
    }
  }
}

// Rate records of the kinematic time step (largest sum_k |u0_k| over the
// workgroup's nodes), one thread per node.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_kin1_rate(long long n, const double* __restrict__ u0,
                                                     double* __restrict__ rec) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  double w = 0.0;
  if (i < n) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) w += fabs(u0[k * n + i]);
  }
  block_rate_record(w, 0.0, rec, blockIdx.x);
}

// Per-workgroup sums of W |phi - phi0|, W (phi - phi0), W phi0 with the p = 1
// GLL weights (1 per axis): W = prod_k J_k.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_kin1_errors(KArgs A, long long n, const double* __restrict__ phi,
                                                       const double* __restrict__ phi0, double* __restrict__ rec) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  double v[KERR] = {0.0, 0.0, 0.0, 0.0};
  if (i < n) {
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) W *= A.J[k];
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

}  // namespace dg2p

namespace dg2p {

// Velocity amplitude from a nodal stream function S (2D, either order):
// u0 = (dS/dy, -dS/dx) with the element-local nodal derivatives, one thread
// per node.  D is the GLL derivative matrix of the mesh's order (n x n used).
struct CurlArgs {
  double D[4][4];
  double Jinv[2];
  int n;
  long long E;
};

__global__ __launch_bounds__(BLOCK) void k_kin_curl(CurlArgs C, const double* __restrict__ S,
                                                    double* __restrict__ u0) {
  const int n = C.n, nn = n * n;
  const long long total = C.E * nn;
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= total) return;
  const long long e = i / nn;
  const int j = (int)(i - e * nn);
  const int ax = j % n, ay = j / n;
  const double* s = S + e * nn;
  double dx = 0.0, dy = 0.0;
  for (int b = 0; b < n; ++b) {
    dx = fma(C.D[ax][b], s[b + n * ay], dx);
    dy = fma(C.D[ay][b], s[ax + n * b], dy);
  }
  u0[i] = dy * C.Jinv[1];
  u0[total + i] = -(dx * C.Jinv[0]);
}

}  // namespace dg2p
