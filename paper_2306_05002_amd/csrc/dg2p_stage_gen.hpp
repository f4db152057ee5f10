// Quadrilaterals of a general degree P (the paper's p = 4 runs of the
// Rayleigh-Taylor instability and the rising bubble, Results, "Two-phase
// flows"): the same residual, stage combination, face ingredients and records
// as k_stage / k_ingredients / k_records, for (P+1)^2 nodes per element.
//
// Lane map: one lane per GLL node, two elements per wave (lanes 0..NN-1 and
// 32..32+NN-1, NN = (P+1)^2 <= 32), one-wave workgroups.  Node j = a_x +
// (P+1) a_y.  Derivatives go through an LDS tile of the element: the lanes
// write the values to differentiate, the workgroup barrier (one wave) makes
// them visible, and each lane sums its P+1 line neighbours with its rows of D
// (the DPP lane maps of the p = 3 kernels are tied to four nodes per line).
// The node-level arithmetic (closure, fluxes, face fluxes with every boundary
// ghost, time-step and monitor records) is the p = 3 kernels' own functions.
// FP64 only; the host selects these kernels for order != 3 in 2D.

#pragma once

#include "dg2p_device.hpp"

namespace dg2p {

template <int P>
struct GenLane {
  static constexpr int NP = P + 1;
  static constexpr int NN = NP * NP;
  static_assert(NN <= 32, "two elements per wave");
  int half;      // which element of the wave
  int slot;      // lane within the element's half (>= NN: no node)
  int node;      // node index (0 for a lane without node)
  int ax, ay;    // GLL indices of the node
  bool active;   // lane carries a node
  double d[2][NP];  // D[a_k][b] / J_k, k = x, y
};

// Entry (i, b) of the host-built GLL derivative table, for a per-lane i, by
// selects among the kernel-argument values (no indexed argument load).
template <int P>
__device__ __forceinline__ double gen_D(const KArgs& A, int i, int b) {
  double v = A.gD[0][b];
#pragma unroll
  for (int a = 1; a <= P; ++a) v = (i == a) ? A.gD[a][b] : v;
  return v;
}
template <int P>
__device__ __forceinline__ double gen_w(const KArgs& A, int i) {
  double v = A.gw[0];
#pragma unroll
  for (int a = 1; a <= P; ++a) v = (i == a) ? A.gw[a] : v;
  return v;
}

template <int P>
__device__ __forceinline__ void gen_setup(const KArgs& A, GenLane<P>& G) {
  const int lane = threadIdx.x & 63;
  G.half = lane >> 5;
  G.slot = lane & 31;
  G.active = G.slot < GenLane<P>::NN;
  G.node = G.active ? G.slot : 0;
  G.ax = G.node % (P + 1);
  G.ay = G.node / (P + 1);
#pragma unroll
  for (int b = 0; b <= P; ++b) {
    G.d[0][b] = gen_D<P>(A, G.ax, b) * A.Jinv[0];
    G.d[1][b] = gen_D<P>(A, G.ay, b) * A.Jinv[1];
  }
}

// Tile of NV values per lane: tile[half][v][slot].
template <int NV>
struct GenTile {
  double t[2][NV][32];
};

// Writes NV values of every lane to the tile and waits for the workgroup.
template <int P, int NV>
__device__ __forceinline__ void gen_put(GenTile<NV>& T, const GenLane<P>& G, const double* v) {
  __syncthreads();  // earlier reads of the tile are done
#pragma unroll
  for (int i = 0; i < NV; ++i) T.t[G.half][i][G.slot] = v[i];
  __syncthreads();
}

// Derivative along k of tile value i at the lane's node.
template <int P, int NV>
__device__ __forceinline__ double gen_dk(const GenTile<NV>& T, const GenLane<P>& G, int i, int k) {
  constexpr int NP = P + 1;
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int idx = k == 0 ? (G.ay * NP + b) : (b * NP + G.ax);
    s = fma(G.d[k][b], T.t[G.half][i][idx], s);
  }
  return s;
}

// Value i of the tile at node idx of the lane's element.
template <int NV>
__device__ __forceinline__ double gen_at(const GenTile<NV>& T, int half, int i, int idx) {
  return T.t[half][i][idx];
}

// Gradient quantities of a node (the quantities of gradients() for 2D).
template <int P, bool VISC>
__device__ __forceinline__ void gen_gradients(const KArgs& A, const double* q, const Prim& p, const GenLane<P>& G,
                                              Grad<2, VISC>& g) {
  constexpr int NV = VISC ? 4 : 2;
  __shared__ GenTile<NV> T;
  const double al = q[5], ps = q[6];
  double v[NV];
  v[0] = al;
  v[1] = ps;
  if constexpr (VISC) {
    v[2] = p.u[0];
    v[3] = p.u[1];
  }
  gen_put<P, NV>(T, G, v);
  double gP[2];
  double g2 = 0.0;
  g.upsi = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    g.gA[k] = gen_dk<P, NV>(T, G, 0, k);
    gP[k] = gen_dk<P, NV>(T, G, 1, k);
    g2 = fma(gP[k], gP[k], g2);
    g.upsi = fma(p.u[k], gP[k], g.upsi);
  }
  const double inv = rsqrt_nr(g2 + A.delta * A.delta);
  const double aa = al * (1.0 - al);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    g.nh[k] = gP[k] * inv;
    g.a[k] = A.Gamma * (A.eps * g.gA[k] - aa * g.nh[k]);
  }
  if constexpr (VISC) {
    double gU[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) gU[j][k] = gen_dk<P, NV>(T, G, 2 + j, k);
    const double div = gU[0][0] + gU[1][1];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) g.S[j][k] = gU[j][k] + gU[k][j] - (j == k ? (2.0 / 3.0) * div : 0.0);
    g.mu = A.mu1 * al + A.mu2 * (1.0 - al);
  } else {
    g.mu = 0.0;
  }
}

// Face ingredients of the state q (a.e_k and the viscous traction at the
// element's face nodes) into G, and its records (REC_MODE 1: rate, 2: all).
template <int P, bool VISC, bool WRITE_G, int REC_MODE>
__device__ __forceinline__ void gen_emit(const KArgs& A, const double* q, long long e, bool valid,
                                         const GenLane<P>& Gl, double* G, double* rec, long long blk,
                                         double* rate = nullptr) {
  constexpr int C = VISC ? 3 : 1;
  constexpr int NFN = P + 1;
  Prim p;
  closure<2>(A, q, p);
  if constexpr (WRITE_G) {
    Grad<2, VISC> g;
    gen_gradients<P, VISC>(A, q, p, Gl, g);
    if (valid) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int ak = k == 0 ? Gl.ax : Gl.ay;
        if (ak != 0 && ak != P) continue;
        const int side = ak == P;
        const int fn = k == 0 ? Gl.ay : Gl.ax;
        const long long base = (long long)((2 * k + side) * C) * A.E;
        G[(base + e) * NFN + fn] = g.a[k];
        if constexpr (VISC) {
#pragma unroll
          for (int j = 0; j < 2; ++j) G[(base + (long long)(1 + j) * A.E + e) * NFN + fn] = g.mu * g.S[j][k];
        }
      }
    }
  }
  if constexpr (REC_MODE == 2) {
    double v[REC];
    const double W = gen_w<P>(A, Gl.ax) * gen_w<P>(A, Gl.ay) * A.J[0] * A.J[1];
    node_record_w<2, VISC>(A, q, p, W, valid, v);
    block_record<64>(v, rec, blk, rate);
  } else if constexpr (REC_MODE == 1) {
    double w = 2.0 * p.c + fabs(p.u[0]) + fabs(p.u[1]);
    double nu = 0.0;
    if constexpr (VISC) {
      const double al = q[5];
      nu = (A.mu1 * al + A.mu2 * (1.0 - al)) * rcp_nr(p.rho);
    }
    block_rate_record<64>(valid ? w : 0.0, valid ? nu : 0.0, rec, blk);
  }
}

// Element and node of a lane in logical block blk (two elements per
// workgroup).
template <int P>
__device__ __forceinline__ long long gen_elem(const KArgs& A, long long blk, const GenLane<P>& G, bool& valid) {
  const long long e0 = blk * 2 + G.half;
  valid = G.active && e0 < A.E;
  return e0 < A.E ? e0 : A.E - 1;
}

template <int P, bool VISC>
__global__ __launch_bounds__(64) void k_ingredients_g(KArgs A, const double* __restrict__ U, double* __restrict__ G,
                                                      double* __restrict__ rec) {
  constexpr int NN = (P + 1) * (P + 1);
  const long long blk = logical_block(A);
  if (blk < 0) return;
  GenLane<P> Gl;
  gen_setup<P>(A, Gl);
  bool valid;
  const long long e = gen_elem<P>(A, blk, Gl, valid);
  double q[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) q[f] = U[(f * A.E + e) * NN + Gl.node];
  gen_emit<P, VISC, true, 1>(A, q, e, valid, Gl, G, rec, blk);
}

// Stage pass (modes, epilogues and the fused time step and monitors of a
// small grid as k_stage).
template <int P, bool VISC, bool CSF, int BCK, int MODE, int EPI>
__global__ __launch_bounds__(64) void k_stage_g(KArgs A, StageIO io) {
  constexpr int NP = P + 1;
  constexpr int NN = NP * NP;
  constexpr int NFN = NP;
  constexpr int NF = 7, NC = 5;
  constexpr int C = VISC ? 3 : 1;
  const long long blk = logical_block(A);
  if (blk < 0) return;
  GenLane<P> Gl;
  gen_setup<P>(A, Gl);
  bool valid;
  const long long e = gen_elem<P>(A, blk, Gl, valid);
  const double* __restrict__ Us = io.Us;
  double q[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) q[f] = Us[(f * A.E + e) * NN + Gl.node];
  double dt_in = 0.0;
  if constexpr (MODE != 0) {
    if (!(MODE == 1 && io.dt_out)) dt_in = *io.dt;
  }
  // first stage of a small grid: the rate records of the time step
  __shared__ double dt_lds[2][1];
  if constexpr (MODE == 1) {
    if (io.dt_out && (!io.dt_fixed || io.mon_out)) fused_dt_load<64>(A, io.rate_in, dt_lds);
  }
  Prim pr;
  closure<2>(A, q, pr);
  Grad<2, VISC> g;
  gen_gradients<P, VISC>(A, q, pr, Gl, g);

  // volume terms: R_q = sum_k d_k (-F_q + s_q a + V_q)_k, div a - u.grad alpha,
  // -u.grad psi; CSF curvature -div n
  constexpr int NV = 2 * (NC + 1) + (CSF ? 2 : 0);
  __shared__ GenTile<NV> T;
  double vals[NV];
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) {
    const double sq = s_coef<2>(A, pr, qi);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double fl = fma(sq, g.a[k], -conv_flux<2>(q, pr, qi, k));
      if constexpr (VISC) {
        if (qi >= 2 && qi < 4) {
          fl = fma(g.mu, g.S[qi - 2][k], fl);
        } else if (qi == 4) {
          double tu = 0.0;
#pragma unroll
          for (int j = 0; j < 2; ++j) tu = fma(g.S[j][k], pr.u[j], tu);
          fl = fma(g.mu, tu, fl);
        }
      }
      vals[2 * qi + k] = fl;
    }
  }
  vals[2 * NC] = g.a[0];
  vals[2 * NC + 1] = g.a[1];
  if constexpr (CSF) {
    vals[2 * NC + 2] = g.nh[0];
    vals[2 * NC + 3] = g.nh[1];
  }
  gen_put<P, NV>(T, Gl, vals);
  double R[NF];
#pragma unroll
  for (int qi = 0; qi < NC; ++qi) R[qi] = gen_dk<P, NV>(T, Gl, 2 * qi, 0) + gen_dk<P, NV>(T, Gl, 2 * qi + 1, 1);
  {
    const double diva = gen_dk<P, NV>(T, Gl, 2 * NC, 0) + gen_dk<P, NV>(T, Gl, 2 * NC + 1, 1);
    const double ua = fma(pr.u[1], g.gA[1], pr.u[0] * g.gA[0]);
    R[5] = diva - ua;
    R[6] = -g.upsi;
  }
  {
    double csf = 0.0;
    if constexpr (CSF) {
      const double div = gen_dk<P, NV>(T, Gl, 2 * NC + 2, 0) + gen_dk<P, NV>(T, Gl, 2 * NC + 3, 1);
      const double ga2 = fma(g.gA[1], g.gA[1], g.gA[0] * g.gA[0]);
      const double dG = sqrt_nr(ga2 + A.delta * A.delta) - A.delta;
      csf = A.sigma * (-div) * dG;
    }
    if (A.has_grav || CSF) {
      double ew = 0.0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double sj = pr.rho * A.grav[j];
        double ej = pr.rho * A.grav[j] * pr.u[j];
        if constexpr (CSF) {
          sj += csf * g.nh[j];
          ej += csf * pr.u[j] * g.nh[j];
        }
        R[2 + j] += sj;
        ew += ej;
      }
      R[4] += ew;
    }
  }

  // faces: each lane on a face evaluates its own face node(s)
  long long ec[2];
  elem_coords<2>(A, e, ec);
  double symv[2][NC + 1];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int i = 0; i <= NC; ++i) symv[k][i] = 0.0;
    const int ak = k == 0 ? Gl.ax : Gl.ay;
    if (!Gl.active || (ak != 0 && ak != P)) continue;
    const int side = ak == P;
    long long c = ec[k] + (side ? 1 : -1);
    bool bnd = false;
    if (c < 0 || c >= A.N[k]) {
      if (BCK == 0 || bc_kind(A, k, side) == DG2P_BC_PERIODIC)
        c = (c < 0) ? A.N[k] - 1 : 0;
      else
        bnd = true;
    }
    const long long en = bnd ? e : e + (c - ec[k]) * (k == 0 ? 1LL : (long long)A.N[0]);
    const int facing = k == 0 ? (Gl.ay * NP + (P - Gl.ax)) : ((P - Gl.ay) * NP + Gl.ax);
    const int fn = k == 0 ? Gl.ay : Gl.ax;
    double qn[NF], tn[2] = {0.0, 0.0};
#pragma unroll
    for (int f = 0; f < NF; ++f) qn[f] = Us[(f * A.E + en) * NN + facing];
    const long long gb = (long long)((2 * k + (1 - side)) * C) * A.E;
    const double an = io.Gin[(gb + en) * NFN + fn];
    if constexpr (VISC) {
#pragma unroll
      for (int j = 0; j < 2; ++j) tn[j] = io.Gin[(gb + (long long)(1 + j) * A.E + en) * NFN + fn];
    }
    double Sk[2] = {0.0, 0.0};
    if constexpr (VISC) {
      Sk[0] = g.S[0][k];
      Sk[1] = g.S[1][k];
    }
    double Rc[NF];
    face_flux<2, VISC, BCK>(A, k, side, bnd, qn, an, tn, q, pr, g.a[k], g.mu, Sk, g.gA[k], g.nh[k], Rc, symv[k]);
#pragma unroll
    for (int f = 0; f < NF; ++f) R[f] += Rc[f];
  }
  // SIPG symmetric term along each line: the face nodes' values at the two
  // ends, weighted with D[end][a] / (2 w_a J_k^2)
  {
    __shared__ GenTile<2 * (NC + 1)> S;
    double sv[2 * (NC + 1)];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i <= NC; ++i) sv[k * (NC + 1) + i] = symv[k][i];
    gen_put<P, 2 * (NC + 1)>(S, Gl, sv);
    const double wa[2] = {gen_w<P>(A, Gl.ax), gen_w<P>(A, Gl.ay)};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int ak = k == 0 ? Gl.ax : Gl.ay;
      const double wlo = gen_D<P>(A, 0, ak) / wa[k] * A.hJ2inv[k];
      const double whi = gen_D<P>(A, P, ak) / wa[k] * A.hJ2inv[k];
      const int lo = k == 0 ? Gl.ay * NP : Gl.ax;
      const int hi = k == 0 ? Gl.ay * NP + P : P * NP + Gl.ax;
#pragma unroll
      for (int i = 0; i <= NC; ++i) {
        const double vlo = gen_at(S, Gl.half, k * (NC + 1) + i, lo);
        const double vhi = gen_at(S, Gl.half, k * (NC + 1) + i, hi);
        const int f = (i < NC) ? i : 5;
        R[f] = fma(vlo, wlo, fma(vhi, whi, R[f]));
      }
    }
  }

  // the fused time step of a small grid (uniform branch)
  double dt_fused = 0.0;
  if constexpr (MODE == 1) {
    if (io.dt_out) {
      double rate = 0.0;
      if (!io.dt_fixed || io.mon_out) rate = fused_rate_finish<64>(A, dt_lds, (double)(NP * NP * 2));
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
  const long long o = e * NN + Gl.node;
  const long long fs = A.E * NN;
  if constexpr (MODE == 0) {
    if (valid) {
#pragma unroll
      for (int f = 0; f < NF; ++f) io.Out[f * fs + o] = R[f];
    }
  } else {
    const double dt = (MODE == 1 && io.dt_out) ? dt_fused : dt_in;
    double uo[NF];
    if constexpr (MODE == 1) {
#pragma unroll
      for (int f = 0; f < NF; ++f) uo[f] = fma(dt, R[f], q[f]);
    } else {
#pragma unroll
      for (int f = 0; f < NF; ++f) uo[f] = fma(A.rk_a, io.Un[f * fs + o], A.rk_b * fma(dt, R[f], q[f]));
    }
    if (valid) {
#pragma unroll
      for (int f = 0; f < NF; ++f) io.Out[f * fs + o] = uo[f];
    }
    if constexpr (EPI > 0)
      gen_emit<P, VISC, true, (EPI == 2 ? 2 : (EPI == 3 ? 1 : 0))>(A, uo, e, valid, Gl, io.Gout, io.rec, blk,
                                                                  io.rate_out);
    if constexpr (MODE == 1) {
      if (io.mon_out) fused_monitor_slots<64, NF>(A, io.mon_rec, io.mon_out, blk);
    }
  }
}

// Records of a state (dt / monitor requests), grid-stride over nodes.
template <int P, bool VISC>
__global__ __launch_bounds__(BLOCK) void k_records_g(KArgs A, const double* __restrict__ U,
                                                     double* __restrict__ rec) {
  constexpr int NN = (P + 1) * (P + 1);
  const long long n = A.E * NN;
  double acc[REC];
#pragma unroll
  for (int s = 0; s < REC; ++s) acc[s] = (s == R_AMIN) ? INFINITY : (s == R_AMAX ? -INFINITY : 0.0);
  for (long long base = (long long)blockIdx.x * BLOCK; base < n; base += (long long)gridDim.x * BLOCK) {
    const long long i = base + threadIdx.x;
    const bool valid = i < n;
    const long long ii = valid ? i : 0;
    double q[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) q[f] = U[f * n + ii];
    Prim p;
    closure<2>(A, q, p);
    const int node = (int)(ii % NN);
    const double W = gen_w<P>(A, node % (P + 1)) * gen_w<P>(A, node / (P + 1)) * A.J[0] * A.J[1];
    double v[REC];
    node_record_w<2, VISC>(A, q, p, W, valid, v);
#pragma unroll
    for (int s = 0; s < REC; ++s) acc[s] = rec_combine(s, acc[s], v[s]);
  }
  block_record(acc, rec, blockIdx.x);
}

}  // namespace dg2p
