// Host side of libdg2p: the C ABI declared in include/dg2p.h.
//
// Validation, workspace carving and launch orchestration.  All device work
// is stream-ordered; nothing here synchronises the device or allocates
// device memory.

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/dg2p.h"
#include "dg2p_device.hpp"
#include "dg2p_adjoint.hpp"
#include "dg2p_kinematic.hpp"
#include "dg2p_kinematic_p1.hpp"
#include "dg2p_launch.hpp"

using namespace dg2p;

// Device scratch of dg2p_rk_step_noalloc (callers that cannot allocate device
// memory): a file-scope array that every GPU running the library holds until
// the process ends.  Host code never passes `scratch` itself to a kernel (its
// name is a host-side stand-in); it uses the address hipGetSymbolAddress
// returns on each device (noalloc_scratch below).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

struct dg2p_mesh_s {
  dg2p_mesh_desc desc;
  int dim;
  int N[3];
  long long E;
  int nn, nf, nfn;
  double h[3], J[3];
  double xi[8], w[8], D[8][8];
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return DG2P_OK;
  return fail(DG2P_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// GLL nodes and weights of degree 1, 3 or 4 in closed form, and the Lagrange
// derivative matrix D[a][b] = l_b'(xi_a) from the product rule.
void gll(int p, double* x, double* w, double (*D)[8]) {
  const int n = p + 1;
  if (p == 1) {
    x[0] = -1.0;
    x[1] = 1.0;
    w[0] = w[1] = 1.0;
  } else if (p == 4) {
    const double s = std::sqrt(3.0 / 7.0);
    x[0] = -1.0;
    x[1] = -s;
    x[2] = 0.0;
    x[3] = s;
    x[4] = 1.0;
    w[0] = w[4] = 1.0 / 10.0;
    w[1] = w[3] = 49.0 / 90.0;
    w[2] = 32.0 / 45.0;
  } else {
    const double s = 1.0 / std::sqrt(5.0);
    x[0] = -1.0;
    x[1] = -s;
    x[2] = s;
    x[3] = 1.0;
    w[0] = w[3] = 1.0 / 6.0;
    w[1] = w[2] = 5.0 / 6.0;
  }
  for (int a = 0; a < n; ++a) {
    for (int b = 0; b < n; ++b) {
      if (a == b) {
        double t = 0.0;
        for (int m = 0; m < n; ++m)
          if (m != a) t += 1.0 / (x[a] - x[m]);
        D[a][b] = t;
      } else {
        double num = 1.0, den = 1.0;
        for (int m = 0; m < n; ++m) {
          if (m != b) den *= (x[b] - x[m]);
          if (m != a && m != b) num *= (x[a] - x[m]);
        }
        D[a][b] = num / den;
      }
    }
  }
}

int check_params(const dg2p_mesh_s* m, const dg2p_params* p) {
  if (!p) return fail(DG2P_EINVAL, "params is NULL");
  if (m && m->desc.order != 3) {
    if (m->desc.order != 4 || m->dim != 2)
      return fail(DG2P_EUNSUPPORTED,
                  "the two-phase model is implemented for p = 3, and p = 4 on quadrilaterals (p = 1: kinematic mode only)");
    if (p->precision != DG2P_FP64) return fail(DG2P_EUNSUPPORTED, "p = 4 runs in FP64 only");
  }
  for (int l = 0; l < 2; ++l) {
    if (!(p->gamma[l] > 1.0)) return fail(DG2P_EINVAL, "gamma must be > 1");
    if (!std::isfinite(p->pinf[l]) || !std::isfinite(p->rho0[l]))
      return fail(DG2P_EINVAL, "pinf / rho0 must be finite");
    if (!(p->mu[l] >= 0.0)) return fail(DG2P_EINVAL, "mu must be >= 0");
  }
  if (!(p->Gamma >= 0.0) || !(p->eps > 0.0)) return fail(DG2P_EINVAL, "Gamma >= 0 and eps > 0 required");
  if (!(p->c_ip > 0.0)) return fail(DG2P_EINVAL, "c_ip must be > 0");
  if (!(p->grad_reg >= 0.0)) return fail(DG2P_EINVAL, "grad_reg must be >= 0");
  if (!std::isfinite(p->sigma)) return fail(DG2P_EINVAL, "sigma must be finite");
  if (p->precision < DG2P_FP64 || p->precision > DG2P_MIXED_BF16)
    return fail(DG2P_EINVAL, "unknown precision");
  (void)m;
  return DG2P_OK;
}


// Threads per workgroup of the element passes of a mesh (ewg<DIM>(); the
// quadrilaterals of degree != 3 run one-wave workgroups of two elements).
bool generic_order(const dg2p_mesh_s* m) { return m->desc.order != 3; }
int elem_threads(const dg2p_mesh_s* m) {
  if (generic_order(m) && m->dim == 2) return 64;
  return m->dim == 3 ? ewg<3>() : (m->dim == 2 ? ewg<2>() : ewg<1>());
}
// Elements per wave of the element passes.
int elems_per_wave(const dg2p_mesh_s* m) { return generic_order(m) ? 2 : (64 >> (2 * m->dim)); }

KArgs make_args(const dg2p_mesh_s* m, const dg2p_params* p) {
  KArgs A;
  std::memset(&A, 0, sizeof(A));
  A.E = m->E;
  const long long per_wg = (long long)(elem_threads(m) / 64) * elems_per_wave(m);  // elements per workgroup
  A.nblocks = (m->E + per_wg - 1) / per_wg;
  A.xcd_chunk = (A.nblocks + 7) / 8;
  for (int k = 0; k < 3; ++k) {
    A.N[k] = k < m->dim ? m->N[k] : 1;
    for (int s = 0; s < 2; ++s) {
      A.bc[k][s] = k < m->dim ? m->desc.bc[k][s] : DG2P_BC_PERIODIC;
      A.bc_bits |= (unsigned)A.bc[k][s] << (3 * (2 * k + s));
      for (int f = 0; f < 8; ++f) A.bcs[k][s][f] = m->desc.bc_state[k][s][f];
    }
    const double J = k < m->dim ? m->J[k] : 1.0;
    const double h = k < m->dim ? m->h[k] : 1.0;
    A.Jinv[k] = 1.0 / J;
    A.lift[k] = 1.0 / (m->w[0] * J);
    A.pen[k] = p->c_ip * (double)((m->desc.order + 1) * (m->desc.order + 1)) / h;
    A.J[k] = J;
    A.hJ2inv[k] = 1.0 / (2.0 * J * J);
  }
  const double g1 = p->gamma[0], g2 = p->gamma[1];
  A.xi1 = 1.0 / (g1 - 1.0);
  A.xi2 = 1.0 / (g2 - 1.0);
  A.pi1 = g1 * p->pinf[0] / (g1 - 1.0);
  A.pi2 = g2 * p->pinf[1] / (g2 - 1.0);
  A.gh1 = g1 / (g1 - 1.0);
  A.gh2 = g2 / (g2 - 1.0);
  A.pinf1 = p->pinf[0];
  A.pinf2 = p->pinf[1];
  A.rho01 = p->rho0[0];
  A.rho02 = p->rho0[1];
  A.Gamma = p->Gamma;
  A.eps = p->eps;
  A.GammaEps = p->Gamma * p->eps;
  A.mu1 = p->mu[0];
  A.mu2 = p->mu[1];
  A.sigma = p->sigma;
  A.has_grav = 0;
  for (int k = 0; k < 3; ++k) {
    A.grav[k] = k < m->dim ? p->g[k] : 0.0;
    if (A.grav[k] != 0.0) A.has_grav = 1;
  }
  A.delta = p->grad_reg;
  A.rk_a = 0.0;
  A.rk_b = 1.0;
  for (int a = 0; a <= m->desc.order && a < 8; ++a) {
    A.gw[a] = m->w[a];
    for (int b = 0; b <= m->desc.order && b < 8; ++b) A.gD[a][b] = m->D[a][b];
  }
  return A;
}

// ---- optional kernel timing (benchmarks): library-owned event pairs ----
constexpr int TIMING_SLOTS = 8192;
struct Timing {
  bool on = false;
  int used = 0;
  hipEvent_t start[TIMING_SLOTS];
  hipEvent_t stop[TIMING_SLOTS];
  int kind[TIMING_SLOTS];
  bool created = false;
};
Timing g_timing;

struct TimedLaunch {
  int slot = -1;
  hipStream_t s;
  TimedLaunch(int kind, hipStream_t st) : s(st) {
    if (!g_timing.on || g_timing.used >= TIMING_SLOTS) return;
    slot = g_timing.used++;
    g_timing.kind[slot] = kind;
    (void)hipEventRecord(g_timing.start[slot], s);
  }
  ~TimedLaunch() {
    if (slot >= 0) (void)hipEventRecord(g_timing.stop[slot], s);
  }
};

// A roctx range named after the entry point around each call that launches
// work (shown by rocprofv3 --marker-trace beside the kernels it launched; a
// cheap no-op without a tool attached).
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};
#define DG2P_API_RANGE() ApiRange dg2p_api_range_(__func__)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// FP64 FMA issue-rate calibration: every lane runs CALIB_CHAINS independent
// multiply-add recurrences x <- a x + b (a = 1 - 1e-9, b = 1e-9 keep them
// near 1), enough of them and enough waves to hide the FMA latency; the sum
// is stored only if it equals `never` (never the case; sink is NULL), which
// keeps the chains live.
constexpr int CALIB_CHAINS = 8;
constexpr int CALIB_THREADS = 256;
constexpr int CALIB_WGS = 256 * 16;  // 16 four-wave workgroups per CU
constexpr long long CALIB_ITERS = 4096;
__global__ __launch_bounds__(CALIB_THREADS) void k_fma_calib(long long iters, double a, double b, double never,
                                                              double* sink) {
  double x[CALIB_CHAINS];
#pragma unroll
  for (int i = 0; i < CALIB_CHAINS; ++i) x[i] = 1.0 + 1e-3 * i + 1e-12 * threadIdx.x;
  for (long long it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CALIB_CHAINS; ++i) x[i] = fma(x[i], a, b);
  }
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < CALIB_CHAINS; ++i) sum += x[i];
  if (sum == never && sink) sink[threadIdx.x] = sum;
}

bool viscous(const dg2p_params* p) { return p->mu[0] != 0.0 || p->mu[1] != 0.0; }
// boundary code the stage kernels compile in: 0 = none (periodic mesh), 1 =
// ghosts built from the interior trace (walls, extrapolation), 2 = also those
// that read the side's bc_state (Dirichlet, Riemann)
int bc_class(const dg2p_mesh_s* m) {
  int c = 0;
  for (int k = 0; k < m->dim; ++k)
    for (int s = 0; s < 2; ++s) {
      const int b = m->desc.bc[k][s];
      if (b == DG2P_BC_DIRICHLET || b == DG2P_BC_RIEMANN) c = 2;
      else if (b != DG2P_BC_PERIODIC && c < 1) c = 1;
    }
  return c;
}

size_t g_bytes(const dg2p_mesh_s* m, const dg2p_params* p) {
  // components per face node, stored in pairs when more than one (GLay); the
  // p = 4 kernels use C of them
  const int C = viscous(p) ? 1 + m->dim : 1;
  const int CP = C == 1 ? 1 : 2 * ((C + 1) / 2);
  return align256(sizeof(double) * (size_t)(2 * m->dim) * CP * (size_t)m->E * m->nfn);
}
size_t state_bytes(const dg2p_mesh_s* m) {
  return align256(sizeof(double) * (size_t)m->nf * (size_t)m->E * m->nn);
}
constexpr long long REC2_MAX = 1024;   // second-level records
constexpr long long REC_GRID = 1024;   // workgroups of the stand-alone record pass
long long elem_blocks(const dg2p_mesh_s* m) {
  const long long per = (long long)(elem_threads(m) / 64) * elems_per_wave(m);
  return (m->E + per - 1) / per;
}
size_t rec_bytes(const dg2p_mesh_s* m) {
  long long n = elem_blocks(m);
  if (n < REC_GRID) n = REC_GRID;
  return align256(sizeof(double) * (size_t)REC * (size_t)(n + REC2_MAX)) + 256;
}

struct Work {
  double* G0 = nullptr;
  double* G1 = nullptr;
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* rec = nullptr;
  double* rec2 = nullptr;
  double* dt = nullptr;  // internal device scalar
};

size_t fb_bytes(const dg2p_mesh_s* m, const dg2p_params* p) {
  const int C = viscous(p) ? 1 + m->dim : 1;
  return align256(sizeof(double) * (size_t)(2 * m->dim) * (m->nf + C) * (size_t)m->E * m->nfn);
}
size_t vjp_rec_bytes(const dg2p_mesh_s* m) { return align256(sizeof(double) * (size_t)(elem_blocks(m) + 1)); }

size_t work_bytes(const dg2p_mesh_s* m, const dg2p_params* p, int op) {
  switch (op) {
    case DG2P_OP_RHS_VJP: return g_bytes(m, p) + state_bytes(m) + fb_bytes(m, p) + vjp_rec_bytes(m);
    case DG2P_OP_RK_STEP_VJP:
      return 3 * g_bytes(m, p) + 5 * state_bytes(m) + fb_bytes(m, p) + vjp_rec_bytes(m) + rec_bytes(m);
    case DG2P_OP_RHS: return g_bytes(m, p) + rec_bytes(m);
    case DG2P_OP_RK_STEP: return 2 * g_bytes(m, p) + 2 * state_bytes(m) + rec_bytes(m);
    case DG2P_OP_ADVANCE: return 2 * g_bytes(m, p) + 2 * state_bytes(m) + rec_bytes(m) + 256;
    case DG2P_OP_MAX_DT:
    case DG2P_OP_MONITORS: return rec_bytes(m);
    default: return 0;
  }
}

Work carve(const dg2p_mesh_s* m, const dg2p_params* p, int op, void* work) {
  Work w;
  char* c = static_cast<char*>(work);
  const size_t gb = g_bytes(m, p), sb = state_bytes(m);
  if (op == DG2P_OP_RHS || op == DG2P_OP_RK_STEP || op == DG2P_OP_ADVANCE) {
    w.G0 = reinterpret_cast<double*>(c);
    c += gb;
  }
  if (op == DG2P_OP_RK_STEP || op == DG2P_OP_ADVANCE) {
    w.G1 = reinterpret_cast<double*>(c);
    c += gb;
    w.U1 = reinterpret_cast<double*>(c);
    c += sb;
    w.U2 = reinterpret_cast<double*>(c);
    c += sb;
  }
  w.rec = reinterpret_cast<double*>(c);
  long long n = elem_blocks(m);
  if (n < REC_GRID) n = REC_GRID;
  w.rec2 = w.rec + (size_t)REC * n;
  c += rec_bytes(m);
  if (op == DG2P_OP_ADVANCE) w.dt = reinterpret_cast<double*>(c);
  return w;
}

int check_ws(void* work, size_t need) {
  if (need == 0) return DG2P_OK;
  if (!work) return fail(DG2P_EWORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(work) & 255) return fail(DG2P_EWORKSPACE, "workspace is not 256-byte aligned");
  return DG2P_OK;
}

dim3 elem_grid(const KArgs& A) { return dim3((unsigned)(8 * A.xcd_chunk)); }

template <int PR>
void stage_dim(int dim, int bck, bool visc, bool csf, int mode, int epi, const KArgs& A, const StageIO& io,
               hipStream_t s) {
  if (dim == 1) launch_stage_dp<1, PR>(bck, visc, csf, mode, epi, A, io, s);
  else if (dim == 2) launch_stage_dp<2, PR>(bck, visc, csf, mode, epi, A, io, s);
  else launch_stage_dp<3, PR>(bck, visc, csf, mode, epi, A, io, s);
}

void launch_stage(const dg2p_mesh_s* m, const dg2p_params* p, int mode, int epi, const KArgs& A,
                  const StageIO& io, hipStream_t s) {
  TimedLaunch t(DG2P_K_STAGE, s);
  const bool visc = viscous(p), csf = p->sigma != 0.0;
  const int bck = bc_class(m);
  if (generic_order(m)) {
    launch_stage_gen(m->desc.order, bck, visc, csf, mode, epi, A, io, s);
    return;
  }
  if (p->precision == DG2P_MIXED_FP32) stage_dim<1>(m->dim, bck, visc, csf, mode, epi, A, io, s);
  else if (p->precision == DG2P_MIXED_BF16) stage_dim<2>(m->dim, bck, visc, csf, mode, epi, A, io, s);
  else stage_dim<0>(m->dim, bck, visc, csf, mode, epi, A, io, s);
}

template <int PR>
void ingr_dim(int dim, bool visc, const KArgs& A, const double* U, double* G, double* rec, hipStream_t s) {
  if (dim == 1) launch_ingredients_dp<1, PR>(visc, A, U, G, rec, s);
  else if (dim == 2) launch_ingredients_dp<2, PR>(visc, A, U, G, rec, s);
  else launch_ingredients_dp<3, PR>(visc, A, U, G, rec, s);
}

void launch_ingr(const dg2p_mesh_s* m, const dg2p_params* p, const KArgs& A, const double* U, double* G,
                 double* rec, hipStream_t s) {
  TimedLaunch t(DG2P_K_INGREDIENTS, s);
  const bool v = viscous(p);
  if (generic_order(m)) {
    launch_ingredients_gen(m->desc.order, v, A, U, G, rec, s);
    return;
  }
  if (p->precision == DG2P_MIXED_FP32) ingr_dim<1>(m->dim, v, A, U, G, rec, s);
  else if (p->precision == DG2P_MIXED_BF16) ingr_dim<2>(m->dim, v, A, U, G, rec, s);
  else ingr_dim<0>(m->dim, v, A, U, G, rec, s);
}

void launch_records(const dg2p_mesh_s* m, const dg2p_params* p, const KArgs& A, const double* U, double* rec,
                    hipStream_t s) {
  TimedLaunch t(DG2P_K_RATE, s);
  const bool v = viscous(p);
  long long n = m->E * m->nn;
  long long gb = (n + BLOCK - 1) / BLOCK;
  if (gb > REC_GRID) gb = REC_GRID;
  const dim3 g((unsigned)gb), b(BLOCK);
  if (generic_order(m)) {
    launch_records_gen(m->desc.order, v, (unsigned)gb, A, U, rec, s);
    return;
  }
  if (m->dim == 1) {
    if (v) hipLaunchKernelGGL((k_records<1, true>), g, b, 0, s, A, U, rec);
    else hipLaunchKernelGGL((k_records<1, false>), g, b, 0, s, A, U, rec);
  } else if (m->dim == 2) {
    if (v) hipLaunchKernelGGL((k_records<2, true>), g, b, 0, s, A, U, rec);
    else hipLaunchKernelGGL((k_records<2, false>), g, b, 0, s, A, U, rec);
  } else {
    if (v) hipLaunchKernelGGL((k_records<3, true>), g, b, 0, s, A, U, rec);
    else hipLaunchKernelGGL((k_records<3, false>), g, b, 0, s, A, U, rec);
  }
}

long long records_of_records(const dg2p_mesh_s* m, const dg2p_params* p, int standalone) {
  (void)p;
  if (standalone) {
    long long n = m->E * m->nn;
    long long gb = (n + BLOCK - 1) / BLOCK;
    return gb > REC_GRID ? REC_GRID : gb;
  }
  return elem_blocks(m);
}

double min_h(const dg2p_mesh_s* m) {
  double hmin = m->h[0];
  for (int k = 1; k < m->dim; ++k) hmin = std::fmin(hmin, m->h[k]);
  return hmin;
}

// Reduce n records to dt / monitors (two levels when n is large).
void finalize(const dg2p_mesh_s* m, const KArgs& A, const Work& w, long long n, double cfl, const double* dt_fixed,
              double* dt, double* t, dg2p_monitors* mon, hipStream_t s) {
  TimedLaunch tl(DG2P_K_RATE_FINAL, s);
  const double* src = w.rec;
  if (n > FIN_THREADS) {
    long long chunk = (n + REC2_MAX - 1) / REC2_MAX;
    if (chunk < BLOCK) chunk = BLOCK;
    const long long nb = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_reduce_records<REC>, dim3((unsigned)nb), dim3(BLOCK), 0, s, w.rec, n, chunk, w.rec2);
    src = w.rec2;
    n = nb;
  }
  const double pdim = (double)((m->desc.order + 1) * (m->desc.order + 1) * m->dim);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, s, src, n, A.GammaEps, pdim, m->nf, min_h(m),
                     cfl, dt_fixed, dt, t, mon);
}

// Reduce n rate records (2 doubles each) to *dt (two levels when n is large).
void finalize_rate(const dg2p_mesh_s* m, const KArgs& A, const Work& w, long long n, double cfl,
                   const double* dt_fixed, double* dt, double* t, hipStream_t s) {
  TimedLaunch tl(DG2P_K_RATE_FINAL, s);
  const double* src = w.rec;
  if (n > FIN_THREADS) {
    long long chunk = (n + REC2_MAX - 1) / REC2_MAX;
    if (chunk < BLOCK) chunk = BLOCK;
    const long long nb = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_reduce_records<RATE>, dim3((unsigned)nb), dim3(BLOCK), 0, s, w.rec, n, chunk, w.rec2);
    src = w.rec2;
    n = nb;
  }
  const double pdim = (double)((m->desc.order + 1) * (m->desc.order + 1) * m->dim);
  hipLaunchKernelGGL(k_finalize_rate, dim3(1), dim3(FIN_THREADS), 0, s, src, n, A.GammaEps, pdim, min_h(m), cfl,
                     dt_fixed, dt, t);
}

// Largest number of rate records for which every workgroup of the first stage
// reduces them itself (16 KB per workgroup) instead of a separate reduction.
#ifndef DG2P_FUSED_DT_MAX
#define DG2P_FUSED_DT_MAX 1024
#endif
constexpr long long FUSED_DT_MAX = DG2P_FUSED_DT_MAX;
static_assert(FUSED_DT_MAX <= FUSED_RATE_MAX, "a first-stage workgroup reduces at most FUSED_RATE_MAX records");
static_assert(RATE * FUSED_DT_MAX <= REC * REC2_MAX, "a monitored step's rate copy fits the second-level records");

bool all_periodic(const dg2p_mesh_s* m) {
  for (int k = 0; k < m->dim; ++k)
    if (m->desc.bc[k][0] != DG2P_BC_PERIODIC) return false;
  return true;
}

// Ub (+)= (dR/dU)^T Rb at state U; sigma cotangent added to *sigb when non-NULL.
void residual_vjp(const dg2p_mesh_s* m, const dg2p_params* p, const KArgs& A, const double* U, const double* G,
                  const double* Rb, double* T, double* FB, double* rec, double* Ub, int accumulate, double* sigb,
                  hipStream_t s) {
  const bool visc = viscous(p);
  const bool csf = p->sigma != 0.0 || sigb != nullptr;
  const bool walls = !all_periodic(m);
  VjpIO io{U, G, Rb, T, FB, rec, Ub, accumulate};
  {
    TimedLaunch t(DG2P_K_VJP_LOCAL, s);
    switch (m->dim) {
      case 1: launch_vjp_dim<1>(visc, csf, walls, A, io, s); break;
      case 2: launch_vjp_dim<2>(visc, csf, walls, A, io, s); break;
      default: launch_vjp_dim<3>(visc, csf, walls, A, io, s); break;
    }
  }
  if (sigb && csf) hipLaunchKernelGGL(k_sum_add, dim3(1), dim3(BLOCK), 0, s, rec, A.nblocks, sigb);
}

// ---- kinematic mode ------------------------------------------------------------

int check_kin(const dg2p_mesh_s* m, const dg2p_kin_params* kp) {
  if (!kp) return fail(DG2P_EINVAL, "kinematic params is NULL");
  if (!(kp->Gamma >= 0.0) || !(kp->eps > 0.0)) return fail(DG2P_EINVAL, "Gamma >= 0 and eps > 0 required");
  if (!(kp->c_ip > 0.0)) return fail(DG2P_EINVAL, "c_ip must be > 0");
  if (!(kp->grad_reg >= 0.0)) return fail(DG2P_EINVAL, "grad_reg must be >= 0");
  if (!std::isfinite(kp->period)) return fail(DG2P_EINVAL, "period must be finite");
  if (!all_periodic(m)) return fail(DG2P_EUNSUPPORTED, "the kinematic mode supports periodic meshes only");
  if (m->desc.order != 1 && m->desc.order != 3) return fail(DG2P_EUNSUPPORTED, "the kinematic mode runs p = 1 or 3");
  return DG2P_OK;
}

KArgs kin_args(const dg2p_mesh_s* m, const dg2p_kin_params* kp) {
  dg2p_params p;
  std::memset(&p, 0, sizeof(p));
  p.gamma[0] = p.gamma[1] = 2.0;  // closure constants unused by the kinematic kernels
  p.Gamma = kp->Gamma;
  p.eps = kp->eps;
  p.c_ip = kp->c_ip;
  p.grad_reg = kp->grad_reg;
  return make_args(m, &p);
}

constexpr double PI = 3.141592653589793;
double kin_factor(const dg2p_kin_params* kp, double t) {
  return kp->period > 0.0 ? std::cos(PI * t / kp->period) : 1.0;
}

size_t kin_state_bytes(const dg2p_mesh_s* m) { return align256(sizeof(double) * 2 * (size_t)m->E * m->nn); }
size_t kin_g_bytes(const dg2p_mesh_s* m) {
  return align256(sizeof(double) * (size_t)(2 * m->dim) * (size_t)m->E * m->nfn);
}
long long kin_err_blocks(const dg2p_mesh_s* m) { return (m->E * m->nn + BLOCK - 1) / BLOCK; }
size_t kin_aux_bytes(const dg2p_mesh_s* m) {
  long long n = elem_blocks(m) * RATE;
  const long long ne = kin_err_blocks(m) * KERR;
  if (ne > n) n = ne;
  return align256(sizeof(double) * (size_t)(n + RATE * REC2_MAX)) + 256;
}
size_t kin_work_bytes(const dg2p_mesh_s* m, int op) {
  switch (op) {
    case DG2P_OP_KIN_RHS: return kin_g_bytes(m);
    case DG2P_OP_KIN_RK4: return 2 * kin_g_bytes(m) + 3 * kin_state_bytes(m) + kin_state_bytes(m) / 2 + 256;
    case DG2P_OP_KIN_AUX: return kin_aux_bytes(m);
    default: return 0;
  }
}

template <int DIM>
void kin_ingr_d(const KArgs& A, const double* P, double* G, hipStream_t s) {
  TimedLaunch t(DG2P_K_INGREDIENTS, s);
  hipLaunchKernelGGL(k_kin_ingredients<DIM>, elem_grid(A), dim3(ewg<DIM>()), 0, s, A, P, G);
}
void kin_ingr(const dg2p_mesh_s* m, const KArgs& A, const double* P, double* G, hipStream_t s) {
  if (m->desc.order == 1) return;  // the p = 1 kernels differentiate the neighbours themselves
  if (m->dim == 1) kin_ingr_d<1>(A, P, G, s);
  else if (m->dim == 2) kin_ingr_d<2>(A, P, G, s);
  else kin_ingr_d<3>(A, P, G, s);
}
template <int DIM>
void kin_stage_d(int mode, const KArgs& A, const KinIO& io, hipStream_t s) {
  TimedLaunch t(DG2P_K_KIN_STAGE, s);
  const dim3 g = elem_grid(A), b(ewg<DIM>());
  if (mode == 0) hipLaunchKernelGGL((k_kin_stage<DIM, 0>), g, b, 0, s, A, io);
  else if (mode == 1) hipLaunchKernelGGL((k_kin_stage<DIM, 1>), g, b, 0, s, A, io);
  else hipLaunchKernelGGL((k_kin_stage<DIM, 2>), g, b, 0, s, A, io);
}
template <int DIM>
void kin1_stage_d(int mode, const KArgs& A, const KinIO& io, hipStream_t s) {
  TimedLaunch t(DG2P_K_KIN_STAGE, s);
  const dim3 g((unsigned)((A.E + BLOCK - 1) / BLOCK)), b(BLOCK);
  if (mode == 0) hipLaunchKernelGGL((k_kin1_stage<DIM, 0>), g, b, 0, s, A, io);
  else if (mode == 1) hipLaunchKernelGGL((k_kin1_stage<DIM, 1>), g, b, 0, s, A, io);
  else hipLaunchKernelGGL((k_kin1_stage<DIM, 2>), g, b, 0, s, A, io);
}
void kin_stage(const dg2p_mesh_s* m, int mode, const KArgs& A, const KinIO& io, hipStream_t s) {
  if (m->desc.order == 1) {
    if (m->dim == 1) kin1_stage_d<1>(mode, A, io, s);
    else if (m->dim == 2) kin1_stage_d<2>(mode, A, io, s);
    else kin1_stage_d<3>(mode, A, io, s);
    return;
  }
  if (m->dim == 1) kin_stage_d<1>(mode, A, io, s);
  else if (m->dim == 2) kin_stage_d<2>(mode, A, io, s);
  else kin_stage_d<3>(mode, A, io, s);
}

template <int DIM>
void reinit_stage_d(int mode, const KArgs& A, const ReinitIO& io, hipStream_t s) {
  TimedLaunch t(DG2P_K_KIN_STAGE, s);
  const dim3 g = elem_grid(A), b(ewg<DIM>());
  if (mode == 1) hipLaunchKernelGGL((k_reinit_stage<DIM, 1>), g, b, 0, s, A, io);
  else hipLaunchKernelGGL((k_reinit_stage<DIM, 2>), g, b, 0, s, A, io);
}
void reinit_stage(const dg2p_mesh_s* m, int mode, const KArgs& A, const ReinitIO& io, hipStream_t s) {
  if (m->dim == 1) reinit_stage_d<1>(mode, A, io, s);
  else if (m->dim == 2) reinit_stage_d<2>(mode, A, io, s);
  else reinit_stage_d<3>(mode, A, io, s);
}

// One SSP-RK3 step with the workspace `work` (carved as for DG2P_OP_RK_STEP).
void rk_step_launch(const dg2p_mesh_s* m, const dg2p_params* p, double* U, const double* dt, void* work,
                    hipStream_t s) {
  KArgs A = make_args(m, p);
  Work w = carve(m, p, DG2P_OP_RK_STEP, work);
  launch_ingr(m, p, A, U, w.G0, w.rec, s);
  // stage 1: U1 = U + dt R(U)
  StageIO io1{U, w.G0, nullptr, w.U1, w.G1, w.rec, dt};
  launch_stage(m, p, 1, 1, A, io1, s);
  // stage 2: U2 = 3/4 U + 1/4 (U1 + dt R(U1))
  A.rk_a = 0.75;
  A.rk_b = 0.25;
  StageIO io2{w.U1, w.G1, U, w.U2, w.G0, w.rec, dt};
  launch_stage(m, p, 2, 1, A, io2, s);
  // stage 3: U <- 1/3 U + 2/3 (U2 + dt R(U2)); each node reads its own U before writing it
  A.rk_a = 1.0 / 3.0;
  A.rk_b = 2.0 / 3.0;
  StageIO io3{w.U2, w.G0, U, U, nullptr, nullptr, dt};
  launch_stage(m, p, 2, 0, A, io3, s);
}

// Per-device address of `scratch`, looked up once per device (with that
// device current) by hipGetSymbolAddress; never the host-side name.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_scratch(void** out) {
  int dev = -1;
  int st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(DG2P_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st) return st;
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255))
      return fail(DG2P_EHIP, "hipGetSymbolAddress(scratch) returned an unusable address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DG2P_OK;
}

}  // namespace

extern "C" {

const char* dg2p_version(void) { return "dg2p 0.2 (gfx950; p = 3, p = 4 on quadrilaterals, p = 1 kinematic)"; }

const char* dg2p_status_string(int status) {
  switch (status) {
    case DG2P_OK: return "DG2P_OK";
    case DG2P_EINVAL: return "DG2P_EINVAL";
    case DG2P_EHIP: return "DG2P_EHIP";
    case DG2P_ENONPHYS: return "DG2P_ENONPHYS";
    case DG2P_EUNSUPPORTED: return "DG2P_EUNSUPPORTED";
    case DG2P_EWORKSPACE: return "DG2P_EWORKSPACE";
    default: return "unknown status";
  }
}

const char* dg2p_last_error(void) { return g_last_error.c_str(); }

int dg2p_create_mesh(const dg2p_mesh_desc* desc, dg2p_mesh* out) {
  g_last_error.clear();
  if (!desc || !out) return fail(DG2P_EINVAL, "desc and out must be non-NULL");
  *out = nullptr;
  if (desc->dim < 1 || desc->dim > 3) return fail(DG2P_EINVAL, "dim must be 1, 2 or 3");
  if (desc->order != 3 && desc->order != 1 && !(desc->order == 4 && desc->dim == 2))
    return fail(DG2P_EUNSUPPORTED,
                "polynomial order 3, 4 on quadrilaterals, and 1 for the kinematic mode are implemented");
  long long E = 1;
  for (int k = 0; k < desc->dim; ++k) {
    if (desc->n_elem[k] < 1) return fail(DG2P_EINVAL, "n_elem must be >= 1");
    if (!(desc->hi[k] > desc->lo[k]) || !std::isfinite(desc->hi[k] - desc->lo[k]))
      return fail(DG2P_EINVAL, "hi must exceed lo");
    for (int s = 0; s < 2; ++s) {
      if (desc->bc[k][s] < DG2P_BC_PERIODIC || desc->bc[k][s] > DG2P_BC_RIEMANN)
        return fail(DG2P_EINVAL, "unknown boundary kind");
      if (desc->bc[k][s] == DG2P_BC_RIEMANN && !(desc->bc_state[k][s][0] > 0.0))
        return fail(DG2P_EINVAL, "Riemann boundary needs a far-field pressure > 0 in bc_state[0]");
    }
    if ((desc->bc[k][0] == DG2P_BC_PERIODIC) != (desc->bc[k][1] == DG2P_BC_PERIODIC))
      return fail(DG2P_EINVAL, "periodic must be set on both sides of an axis");
    // (checked before the product, which could otherwise overflow)
    if (E > (1LL << 40) / desc->n_elem[k]) return fail(DG2P_EINVAL, "mesh too large");
    E *= desc->n_elem[k];
  }
  const int np1 = desc->order + 1;
  long long nn = 1;
  for (int k = 0; k < desc->dim; ++k) nn *= np1;
  if (E > (1LL << 40) / nn) return fail(DG2P_EINVAL, "mesh too large");
  // element indices are formed in 32 bits inside the kernels
  if (E >= (1LL << 31)) return fail(DG2P_EINVAL, "mesh has 2^31 or more elements");
  dg2p_mesh_s* m = new dg2p_mesh_s;
  std::memset(m, 0, sizeof(*m));
  m->desc = *desc;
  m->dim = desc->dim;
  m->E = E;
  m->nn = (int)nn;
  m->nf = desc->dim + 5;
  m->nfn = (int)(nn / np1);
  for (int k = 0; k < 3; ++k) {
    m->N[k] = k < desc->dim ? desc->n_elem[k] : 1;
    m->h[k] = k < desc->dim ? (desc->hi[k] - desc->lo[k]) / desc->n_elem[k] : 1.0;
    m->J[k] = 0.5 * m->h[k];
  }
  gll(desc->order, m->xi, m->w, m->D);
  *out = m;
  return DG2P_OK;
}

int dg2p_destroy_mesh(dg2p_mesh m) {
  delete m;
  return DG2P_OK;
}

int dg2p_layout(dg2p_mesh m, int* n_fields, long long* n_elem, int* nodes_per_elem) {
  if (!m) return fail(DG2P_EINVAL, "mesh is NULL");
  if (n_fields) *n_fields = m->nf;
  if (n_elem) *n_elem = m->E;
  if (nodes_per_elem) *nodes_per_elem = m->nn;
  return DG2P_OK;
}

int dg2p_node_coords(dg2p_mesh m, double* xyz) {
  if (!m || !xyz) return fail(DG2P_EINVAL, "mesh and xyz must be non-NULL");
  const long long E = m->E;
  for (int k = 0; k < m->dim; ++k) {
    long long stride = 1;
    for (int kk = 0; kk < k; ++kk) stride *= m->N[kk];
    for (long long e = 0; e < E; ++e) {
      const long long ek = (e / stride) % m->N[k];
      for (int j = 0; j < m->nn; ++j) {
        int a = j;
        for (int kk = 0; kk < k; ++kk) a /= (m->desc.order + 1);
        a %= (m->desc.order + 1);
        xyz[((long long)k * E + e) * m->nn + j] =
            m->desc.lo[k] + m->h[k] * (double)ek + m->J[k] * (m->xi[a] + 1.0);
      }
    }
  }
  return DG2P_OK;
}

int dg2p_workspace_size(dg2p_mesh m, const dg2p_params* p, int op, size_t* bytes) {
  if (!m || !bytes) return fail(DG2P_EINVAL, "mesh and bytes must be non-NULL");
  int st = check_params(m, p);
  if (st) return st;
  switch (op) {
    case DG2P_OP_RHS:
    case DG2P_OP_RK_STEP:
    case DG2P_OP_ADVANCE:
    case DG2P_OP_MAX_DT:
    case DG2P_OP_MONITORS:
    case DG2P_OP_RHS_VJP:
    case DG2P_OP_RK_STEP_VJP: *bytes = work_bytes(m, p, op); break;
    default: return fail(DG2P_EINVAL, "unknown operation");
  }
  return DG2P_OK;
}

int dg2p_prim_to_cons(dg2p_mesh m, const dg2p_params* p, const double* prim, double* U, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !prim || !U) return fail(DG2P_EINVAL, "mesh, prim and U must be non-NULL");
  if (prim == U) return fail(DG2P_EINVAL, "prim and U may not alias");
  int st = check_params(m, p);
  if (st) return st;
  KArgs A = make_args(m, p);
  const long long n = m->E * m->nn;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipStream_t s = (hipStream_t)stream;
  TimedLaunch t(DG2P_K_PRIM, s);
  switch (m->dim) {
    case 1: hipLaunchKernelGGL((k_prim_to_cons<1>), dim3(blocks), dim3(256), 0, s, A, prim, U, n); break;
    case 2: hipLaunchKernelGGL((k_prim_to_cons<2>), dim3(blocks), dim3(256), 0, s, A, prim, U, n); break;
    default: hipLaunchKernelGGL((k_prim_to_cons<3>), dim3(blocks), dim3(256), 0, s, A, prim, U, n); break;
  }
  return hip_check(hipGetLastError(), "prim_to_cons launch");
}

int dg2p_prim_to_cons_vjp(dg2p_mesh m, const dg2p_params* p, const double* prim, const double* U_bar,
                          double* prim_bar, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !prim || !U_bar || !prim_bar) return fail(DG2P_EINVAL, "mesh, prim, U_bar and prim_bar must be non-NULL");
  if (prim_bar == prim || prim_bar == U_bar) return fail(DG2P_EINVAL, "prim_bar may not alias");
  int st = check_params(m, p);
  if (st) return st;
  KArgs A = make_args(m, p);
  const long long n = m->E * m->nn;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipStream_t s = (hipStream_t)stream;
  switch (m->dim) {
    case 1: hipLaunchKernelGGL((k_prim_to_cons_vjp<1>), dim3(blocks), dim3(256), 0, s, A, prim, U_bar, prim_bar, n); break;
    case 2: hipLaunchKernelGGL((k_prim_to_cons_vjp<2>), dim3(blocks), dim3(256), 0, s, A, prim, U_bar, prim_bar, n); break;
    default: hipLaunchKernelGGL((k_prim_to_cons_vjp<3>), dim3(blocks), dim3(256), 0, s, A, prim, U_bar, prim_bar, n); break;
  }
  return hip_check(hipGetLastError(), "prim_to_cons_vjp launch");
}

int dg2p_node_weights(dg2p_mesh m, double* W) {
  if (!m || !W) return fail(DG2P_EINVAL, "mesh and W must be non-NULL");
  for (int j = 0; j < m->nn; ++j) {
    double w = 1.0;
    int r = j;
    for (int k = 0; k < m->dim; ++k) {
      w *= m->w[r % (m->desc.order + 1)] * m->J[k];
      r /= (m->desc.order + 1);
    }
    W[j] = w;
  }
  return DG2P_OK;
}

int dg2p_rhs(dg2p_mesh m, const dg2p_params* p, const double* U, double* R, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || !R) return fail(DG2P_EINVAL, "mesh, U and R must be non-NULL");
  if (U == R) return fail(DG2P_EINVAL, "U and R may not alias");
  int st = check_params(m, p);
  if (st) return st;
  st = check_ws(work, work_bytes(m, p, DG2P_OP_RHS));
  if (st) return st;
  KArgs A = make_args(m, p);
  Work w = carve(m, p, DG2P_OP_RHS, work);
  hipStream_t s = (hipStream_t)stream;
  launch_ingr(m, p, A, U, w.G0, w.rec, s);
  StageIO io{U, w.G0, nullptr, R, nullptr, nullptr, nullptr};
  launch_stage(m, p, 0, 0, A, io, s);
  return hip_check(hipGetLastError(), "rhs launch");
}

int dg2p_max_dt(dg2p_mesh m, const dg2p_params* p, const double* U, double cfl, double* dt,
                dg2p_monitors* mon, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || (!dt && !mon)) return fail(DG2P_EINVAL, "mesh, U and one of dt/mon must be non-NULL");
  if (!(cfl > 0.0)) return fail(DG2P_EINVAL, "cfl must be > 0");
  int st = check_params(m, p);
  if (st) return st;
  st = check_ws(work, work_bytes(m, p, DG2P_OP_MAX_DT));
  if (st) return st;
  KArgs A = make_args(m, p);
  Work w = carve(m, p, DG2P_OP_MAX_DT, work);
  hipStream_t s = (hipStream_t)stream;
  launch_records(m, p, A, U, w.rec, s);
  finalize(m, A, w, records_of_records(m, p, 1), cfl, nullptr, dt, nullptr, mon, s);
  return hip_check(hipGetLastError(), "max_dt launch");
}

int dg2p_rk_step(dg2p_mesh m, const dg2p_params* p, double* U, const double* dt, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || !dt) return fail(DG2P_EINVAL, "mesh, U and dt must be non-NULL");
  int st = check_params(m, p);
  if (st) return st;
  st = check_ws(work, work_bytes(m, p, DG2P_OP_RK_STEP));
  if (st) return st;
  rk_step_launch(m, p, U, dt, work, (hipStream_t)stream);
  return hip_check(hipGetLastError(), "rk_step launch");
}

int dg2p_rk_step_noalloc(dg2p_mesh m, const dg2p_params* p, double* U, const double* dt, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || !dt) return fail(DG2P_EINVAL, "mesh, U and dt must be non-NULL");
  int st = check_params(m, p);
  if (st) return st;
  const size_t need = work_bytes(m, p, DG2P_OP_RK_STEP);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(DG2P_EWORKSPACE, "dg2p_rk_step_noalloc: this mesh needs " + std::to_string(need) +
                                     " bytes of scratch; the library's static scratch holds " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES) + " (use dg2p_rk_step with a workspace)");
  void* work = nullptr;
  st = noalloc_scratch(&work);
  if (st) return st;
  rk_step_launch(m, p, U, dt, work, (hipStream_t)stream);
  return hip_check(hipGetLastError(), "rk_step_noalloc launch");
}

size_t dg2p_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

}  // extern "C"

namespace {

// n_steps SSP-RK3 steps in place.  Without per-step monitors (mon_steps ==
// NULL) the last stage of every step writes 2-double rate records, from which
// the next step's dt is reduced inside its first stage (small grids) or by
// two small kernels; with them, the last stage writes the full 16-slot
// records, from which the next step's first stage (small grids of at least
// MON_SLOTS workgroups: a copy of their rate slots in rec2 gives dt, the first
// MON_SLOTS workgroups reduce one other slot each) or one reduction per step
// (two small kernels) yields the step's monitors and the next dt; the last
// step's monitors always come from the latter.
int advance_impl(const dg2p_mesh_s* m, const dg2p_params* p, double* U, int n_steps, double cfl,
                 const double* dt_fixed, double* t, double* dt_last, dg2p_monitors* mon, dg2p_monitors* mon_steps,
                 double p_ref, const double* u_ref, void* work, hipStream_t s) {
  KArgs A = make_args(m, p);
  A.p_ref = p_ref;
  if (u_ref)
    for (int k = 0; k < m->dim; ++k) A.u_ref[k] = u_ref[k];
  Work w = carve(m, p, DG2P_OP_ADVANCE, work);
  double* dts = dt_last ? dt_last : w.dt;
  double* Ga = w.G0;
  double* Gb = w.G1;
  // records (rate-only or full) of the ingredient pass and of every step's
  // last stage, one per workgroup
  const long long nrec = elem_blocks(m);
  // a first-stage workgroup reduces up to FUSED_RATE_PER_THREAD records per thread
  const long long fused_max = std::min<long long>(FUSED_DT_MAX, (long long)FUSED_RATE_PER_THREAD * elem_threads(m));
  // (with per-step monitors, a grid of fewer than MON_SLOTS workgroups takes
  // the separate reduction: its workgroups would reduce several slots each)
  const bool fused = nrec <= fused_max && (!mon_steps || nrec >= MON_SLOTS);
  A.cfl = cfl;
  A.hmin = min_h(m);
  A.nrate = nrec;
  launch_ingr(m, p, A, U, Ga, w.rec, s);
  for (int it = 0; it < n_steps; ++it) {
    const bool mon_prev = mon_steps && it > 0;  // monitors of the state after step it - 1
    if (!fused) {
      if (mon_prev) finalize(m, A, w, nrec, cfl, dt_fixed, dts, t, mon_steps + (it - 1), s);
      else finalize_rate(m, A, w, nrec, cfl, dt_fixed, dts, t, s);
    }
    KArgs B = A;
    StageIO io1{U, Ga, nullptr, w.U1, Gb, nullptr, dts};
    if (fused) {
      // rate records: the ingredient pass's in rec, a monitored step's copy in rec2
      io1.rate_in = mon_prev ? w.rec2 : w.rec;
      io1.dt_out = dts;
      io1.t = t;
      io1.dt_fixed = dt_fixed;
      if (mon_prev) {
        io1.mon_rec = w.rec;
        io1.mon_out = mon_steps + (it - 1);
      }
    }
    launch_stage(m, p, 1, 1, B, io1, s);
    B.rk_a = 0.75;
    B.rk_b = 0.25;
    StageIO io2{w.U1, Gb, U, w.U2, Ga, nullptr, dts};
    launch_stage(m, p, 2, 1, B, io2, s);
    B.rk_a = 1.0 / 3.0;
    B.rk_b = 2.0 / 3.0;
    StageIO io3{w.U2, Ga, U, U, Gb, w.rec, dts};
    if (fused && mon_steps) io3.rate_out = w.rec2;
    launch_stage(m, p, 2, mon_steps ? 2 : 3, B, io3, s);
    double* tmp = Ga;
    Ga = Gb;
    Gb = tmp;
  }
  if (mon_steps && n_steps > 0)
    finalize(m, A, w, nrec, cfl, dt_fixed, nullptr, nullptr, mon_steps + (n_steps - 1), s);
  if (mon) {
    // monitors of the final state
    launch_records(m, p, A, U, w.rec, s);
    finalize(m, A, w, records_of_records(m, p, 1), cfl, nullptr, nullptr, nullptr, mon, s);
  }
  return hip_check(hipGetLastError(), "advance launch");
}

int advance_checks(const dg2p_mesh_s* m, const dg2p_params* p, double* U, int n_steps, double cfl,
                   const double* dt_fixed, void* work) {
  if (!m || !U) return fail(DG2P_EINVAL, "mesh and U must be non-NULL");
  if (n_steps < 0) return fail(DG2P_EINVAL, "n_steps must be >= 0");
  if (!dt_fixed && !(cfl > 0.0)) return fail(DG2P_EINVAL, "cfl must be > 0");
  int st = check_params(m, p);
  if (st) return st;
  return check_ws(work, work_bytes(m, p, DG2P_OP_ADVANCE));
}

}  // namespace

extern "C" {

int dg2p_advance(dg2p_mesh m, const dg2p_params* p, double* U, int n_steps, double cfl, const double* dt_fixed,
                 double* t, double* dt_last, dg2p_monitors* mon, double p_ref, const double* u_ref, void* work,
                 void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  int st = advance_checks(m, p, U, n_steps, cfl, dt_fixed, work);
  if (st) return st;
  return advance_impl(m, p, U, n_steps, cfl, dt_fixed, t, dt_last, mon, nullptr, p_ref, u_ref, work,
                      (hipStream_t)stream);
}

int dg2p_advance_monitored(dg2p_mesh m, const dg2p_params* p, double* U, int n_steps, double cfl,
                           const double* dt_fixed, double* t, double* dt_last, dg2p_monitors* mon_steps,
                           double p_ref, const double* u_ref, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!mon_steps) return fail(DG2P_EINVAL, "mon_steps must be non-NULL");
  int st = advance_checks(m, p, U, n_steps, cfl, dt_fixed, work);
  if (st) return st;
  return advance_impl(m, p, U, n_steps, cfl, dt_fixed, t, dt_last, nullptr, mon_steps, p_ref, u_ref, work,
                      (hipStream_t)stream);
}

int dg2p_compute_monitors(dg2p_mesh m, const dg2p_params* p, const double* U, double p_ref, const double* u_ref,
                          dg2p_monitors* mon, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || !mon) return fail(DG2P_EINVAL, "mesh, U and mon must be non-NULL");
  int st = check_params(m, p);
  if (st) return st;
  st = check_ws(work, work_bytes(m, p, DG2P_OP_MONITORS));
  if (st) return st;
  KArgs A = make_args(m, p);
  A.p_ref = p_ref;
  if (u_ref)
    for (int k = 0; k < m->dim; ++k) A.u_ref[k] = u_ref[k];
  Work w = carve(m, p, DG2P_OP_MONITORS, work);
  hipStream_t s = (hipStream_t)stream;
  launch_records(m, p, A, U, w.rec, s);
  finalize(m, A, w, records_of_records(m, p, 1), 0.1, nullptr, nullptr, nullptr, mon, s);
  return hip_check(hipGetLastError(), "monitor launch");
}

int dg2p_rhs_vjp(dg2p_mesh m, const dg2p_params* p, const double* U, const double* R_bar, double* U_bar,
                 double* param_bar, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U || !R_bar || !U_bar) return fail(DG2P_EINVAL, "mesh, U, R_bar and U_bar must be non-NULL");
  if (U_bar == U || U_bar == R_bar) return fail(DG2P_EINVAL, "U_bar may not alias U or R_bar");
  int st = check_params(m, p);
  if (st) return st;
  if (p->precision != DG2P_FP64) return fail(DG2P_EUNSUPPORTED, "the adjoint is FP64 only");
  if (m->desc.order != 3) return fail(DG2P_EUNSUPPORTED, "the adjoint is implemented for p = 3");
  st = check_ws(work, work_bytes(m, p, DG2P_OP_RHS_VJP));
  if (st) return st;
  KArgs A = make_args(m, p);
  char* c = static_cast<char*>(work);
  double* G = reinterpret_cast<double*>(c);
  c += g_bytes(m, p);
  double* T = reinterpret_cast<double*>(c);
  c += state_bytes(m);
  double* FB = reinterpret_cast<double*>(c);
  c += fb_bytes(m, p);
  double* rec = reinterpret_cast<double*>(c);
  hipStream_t s = (hipStream_t)stream;
  // forward face ingredients of U (the neighbours' a.e_k, tau.e_k); its records go to rec2-less scratch: T
  launch_ingr(m, p, A, U, G, T, s);
  residual_vjp(m, p, A, U, G, R_bar, T, FB, rec, U_bar, 0, param_bar, s);
  return hip_check(hipGetLastError(), "rhs_vjp launch");
}

int dg2p_rk_step_vjp(dg2p_mesh m, const dg2p_params* p, const double* U_n, const double* dt, const double* U_np1_bar,
                     double* U_n_bar, double* param_bar, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !U_n || !dt || !U_np1_bar || !U_n_bar)
    return fail(DG2P_EINVAL, "mesh, U_n, dt, U_np1_bar and U_n_bar must be non-NULL");
  if (U_n_bar == U_n || U_n_bar == U_np1_bar) return fail(DG2P_EINVAL, "U_n_bar may not alias U_n or U_np1_bar");
  int st = check_params(m, p);
  if (st) return st;
  if (p->precision != DG2P_FP64) return fail(DG2P_EUNSUPPORTED, "the adjoint is FP64 only");
  if (m->desc.order != 3) return fail(DG2P_EUNSUPPORTED, "the adjoint is implemented for p = 3");
  st = check_ws(work, work_bytes(m, p, DG2P_OP_RK_STEP_VJP));
  if (st) return st;
  KArgs A = make_args(m, p);
  const size_t gb = g_bytes(m, p), sb = state_bytes(m);
  char* c = static_cast<char*>(work);
  double* GA = reinterpret_cast<double*>(c); c += gb;
  double* GB = reinterpret_cast<double*>(c); c += gb;
  double* GC = reinterpret_cast<double*>(c); c += gb;
  double* U1 = reinterpret_cast<double*>(c); c += sb;
  double* U2 = reinterpret_cast<double*>(c); c += sb;
  double* B = reinterpret_cast<double*>(c); c += sb;
  double* Rb = reinterpret_cast<double*>(c); c += sb;
  double* T = reinterpret_cast<double*>(c); c += sb;
  double* FB = reinterpret_cast<double*>(c); c += fb_bytes(m, p);
  double* rec = reinterpret_cast<double*>(c); c += vjp_rec_bytes(m);
  double* rec2 = reinterpret_cast<double*>(c);
  hipStream_t s = (hipStream_t)stream;
  // forward recomputation: U1, U2 and the face ingredients of U_n, U1, U2
  launch_ingr(m, p, A, U_n, GA, rec2, s);
  {
    StageIO io1{U_n, GA, nullptr, U1, GB, nullptr, dt};
    launch_stage(m, p, 1, 1, A, io1, s);
    KArgs B2 = A;
    B2.rk_a = 0.75;
    B2.rk_b = 0.25;
    StageIO io2{U1, GB, U_n, U2, GC, nullptr, dt};
    launch_stage(m, p, 2, 1, B2, io2, s);
  }
  const long long n = (long long)m->nf * m->E * m->nn;
  const unsigned eb = (unsigned)((n + 255) / 256);
  // U3 = 1/3 U + 2/3 (U2 + dt R(U2))
  hipLaunchKernelGGL(k_vjp_combine, dim3(eb), dim3(256), 0, s, n, U_np1_bar, dt, 1.0 / 3.0, 1, U_n_bar, 2.0 / 3.0, B,
                     2.0 / 3.0, Rb);
  residual_vjp(m, p, A, U2, GC, Rb, T, FB, rec, B, 1, param_bar, s);
  // U2 = 3/4 U + 1/4 (U1 + dt R(U1))
  hipLaunchKernelGGL(k_vjp_combine, dim3(eb), dim3(256), 0, s, n, B, dt, 0.75, 0, U_n_bar, 0.25, B, 0.25, Rb);
  residual_vjp(m, p, A, U1, GB, Rb, T, FB, rec, B, 1, param_bar, s);
  // U1 = U + dt R(U)
  hipLaunchKernelGGL(k_vjp_combine, dim3(eb), dim3(256), 0, s, n, B, dt, 1.0, 0, U_n_bar, 0.0, nullptr, 1.0, Rb);
  residual_vjp(m, p, A, U_n, GA, Rb, T, FB, rec, U_n_bar, 1, param_bar, s);
  return hip_check(hipGetLastError(), "rk_step_vjp launch");
}

int dg2p_kin_workspace_size(dg2p_mesh m, int op, size_t* bytes) {
  g_last_error.clear();
  if (!m || !bytes) return fail(DG2P_EINVAL, "mesh and bytes must be non-NULL");
  if (op < DG2P_OP_KIN_RHS || op > DG2P_OP_KIN_AUX) return fail(DG2P_EINVAL, "not a kinematic op");
  *bytes = kin_work_bytes(m, op);
  return DG2P_OK;
}

int dg2p_kin_rhs(dg2p_mesh m, const dg2p_kin_params* kp, const double* Phi, const double* u0, double t, double* R,
                 void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !Phi || !u0 || !R) return fail(DG2P_EINVAL, "mesh, Phi, u0 and R must be non-NULL");
  if (R == Phi) return fail(DG2P_EINVAL, "R may not alias Phi");
  int st = check_kin(m, kp);
  if (st) return st;
  st = check_ws(work, kin_work_bytes(m, DG2P_OP_KIN_RHS));
  if (st) return st;
  const KArgs A = kin_args(m, kp);
  hipStream_t s = (hipStream_t)stream;
  double* G = static_cast<double*>(work);
  kin_ingr(m, A, Phi, G, s);
  KinIO io{};
  io.Ps = Phi;
  io.Gin = G;
  io.u0 = u0;
  io.s = kin_factor(kp, t);
  io.Out = R;
  kin_stage(m, 0, A, io, s);
  return hip_check(hipGetLastError(), "kin_rhs launch");
}

int dg2p_kin_rk4(dg2p_mesh m, const dg2p_kin_params* kp, double* Phi, const double* u0, int n_steps, double t0,
                 double dt, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !Phi || !u0) return fail(DG2P_EINVAL, "mesh, Phi and u0 must be non-NULL");
  if (n_steps < 0) return fail(DG2P_EINVAL, "n_steps must be >= 0");
  if (!std::isfinite(dt) || !std::isfinite(t0)) return fail(DG2P_EINVAL, "t0 and dt must be finite");
  int st = check_kin(m, kp);
  if (st) return st;
  st = check_ws(work, kin_work_bytes(m, DG2P_OP_KIN_RK4));
  if (st) return st;
  const KArgs A = kin_args(m, kp);
  hipStream_t s = (hipStream_t)stream;
  const size_t gb = kin_g_bytes(m), sb = kin_state_bytes(m);
  char* c = static_cast<char*>(work);
  double* G0 = reinterpret_cast<double*>(c); c += gb;
  double* G1 = reinterpret_cast<double*>(c); c += gb;
  double* S1 = reinterpret_cast<double*>(c); c += sb;
  double* S2 = reinterpret_cast<double*>(c); c += sb;
  double* Acc = reinterpret_cast<double*>(c);
  if (n_steps > 0) kin_ingr(m, A, Phi, G0, s);
  for (int it = 0; it < n_steps; ++it) {
    const double t = t0 + it * dt;
    KinIO io{};
    io.u0 = u0;
    io.Pn = Phi;
    io.Acc = Acc;
    // k1 at t: Acc = k1, S1 = Phi + dt/2 k1
    io.Ps = Phi; io.Gin = G0; io.s = kin_factor(kp, t); io.Out = S1; io.Gout = G1;
    io.cdt = 0.5 * dt; io.wacc = 1.0; io.acc_first = 1;
    kin_stage(m, 1, A, io, s);
    // k2 at t + dt/2: Acc += 2 k2, S2 = Phi + dt/2 k2
    io.Ps = S1; io.Gin = G1; io.s = kin_factor(kp, t + 0.5 * dt); io.Out = S2; io.Gout = G0;
    io.cdt = 0.5 * dt; io.wacc = 2.0; io.acc_first = 0;
    kin_stage(m, 1, A, io, s);
    // k3 at t + dt/2: Acc += 2 k3, S1 = Phi + dt k3
    io.Ps = S2; io.Gin = G0; io.Out = S1; io.Gout = G1;
    io.cdt = dt;
    kin_stage(m, 1, A, io, s);
    // k4 at t + dt: Phi += dt/6 (Acc + k4)
    io.Ps = S1; io.Gin = G1; io.s = kin_factor(kp, t + dt); io.Out = Phi; io.Gout = G0;
    io.dt6 = dt / 6.0;
    kin_stage(m, 2, A, io, s);
  }
  return hip_check(hipGetLastError(), "kin_rk4 launch");
}

int dg2p_kin_reinit(dg2p_mesh m, const dg2p_kin_params* kp, double* Phi, int n_iter, double nu, double dtau,
                    void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !Phi) return fail(DG2P_EINVAL, "mesh and Phi must be non-NULL");
  if (n_iter < 0) return fail(DG2P_EINVAL, "n_iter must be >= 0");
  if (!(nu > 0.0) || !std::isfinite(nu) || !std::isfinite(dtau)) return fail(DG2P_EINVAL, "nu > 0, finite dtau");
  int st = check_kin(m, kp);
  if (st) return st;
  if (m->desc.order != 3) return fail(DG2P_EUNSUPPORTED, "the re-initialisation is implemented for p = 3");
  st = check_ws(work, kin_work_bytes(m, DG2P_OP_KIN_RK4));
  if (st) return st;
  // the SIPG coefficient of the diffusive flux is nu: Gamma eps := 1 * nu
  dg2p_kin_params kd = *kp;
  kd.Gamma = 1.0;
  kd.eps = nu;
  const KArgs A = kin_args(m, &kd);
  hipStream_t s = (hipStream_t)stream;
  const size_t gb = kin_g_bytes(m), sb = kin_state_bytes(m);
  char* c = static_cast<char*>(work);
  double* G0 = reinterpret_cast<double*>(c); c += gb;
  double* G1 = reinterpret_cast<double*>(c); c += gb;
  double* S1 = reinterpret_cast<double*>(c); c += sb;
  double* S2 = reinterpret_cast<double*>(c); c += sb;
  double* Acc = reinterpret_cast<double*>(c); c += sb;
  double* sgn = reinterpret_cast<double*>(c);
  double* psi = Phi + (size_t)m->E * m->nn;
  {
    TimedLaunch t(DG2P_K_INGREDIENTS, s);
    if (m->dim == 1)
      hipLaunchKernelGGL(k_reinit_start<1>, elem_grid(A), dim3(ewg<1>()), 0, s, A, Phi, kp->eps, psi, sgn, G0);
    else if (m->dim == 2)
      hipLaunchKernelGGL(k_reinit_start<2>, elem_grid(A), dim3(ewg<2>()), 0, s, A, Phi, kp->eps, psi, sgn, G0);
    else
      hipLaunchKernelGGL(k_reinit_start<3>, elem_grid(A), dim3(ewg<3>()), 0, s, A, Phi, kp->eps, psi, sgn, G0);
  }
  for (int it = 0; it < n_iter; ++it) {
    ReinitIO io{};
    io.sgn = sgn;
    io.Pn = psi;
    io.Acc = Acc;
    io.Ps = psi; io.Gin = G0; io.Out = S1; io.Gout = G1; io.cdt = 0.5 * dtau; io.wacc = 1.0; io.acc_first = 1;
    reinit_stage(m, 1, A, io, s);
    io.Ps = S1; io.Gin = G1; io.Out = S2; io.Gout = G0; io.cdt = 0.5 * dtau; io.wacc = 2.0; io.acc_first = 0;
    reinit_stage(m, 1, A, io, s);
    io.Ps = S2; io.Gin = G0; io.Out = S1; io.Gout = G1; io.cdt = dtau;
    reinit_stage(m, 1, A, io, s);
    io.Ps = S1; io.Gin = G1; io.Out = psi; io.Gout = G0; io.dt6 = dtau / 6.0;
    reinit_stage(m, 2, A, io, s);
  }
  return hip_check(hipGetLastError(), "kin_reinit launch");
}

int dg2p_kin_reinit_params(dg2p_mesh m, double cfl, double* nu, double* dtau) {
  g_last_error.clear();
  if (!m || !nu || !dtau) return fail(DG2P_EINVAL, "mesh, nu and dtau must be non-NULL");
  if (!(cfl > 0.0)) return fail(DG2P_EINVAL, "cfl must be > 0");
  const double hmin = min_h(m);
  const int p = m->desc.order;
  *nu = hmin / (p + 1);
  *dtau = cfl * hmin / (1.0 + (double)((p + 1) * (p + 1) * m->dim) * (*nu) / hmin);
  return DG2P_OK;
}

int dg2p_kin_velocity_from_stream(dg2p_mesh m, const double* S, double* u0, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !S || !u0) return fail(DG2P_EINVAL, "mesh, S and u0 must be non-NULL");
  if (S == u0) return fail(DG2P_EINVAL, "u0 may not alias S");
  if (m->dim != 2) return fail(DG2P_EUNSUPPORTED, "the stream-function velocity is two-dimensional");
  if (m->desc.order != 1 && m->desc.order != 3)
    return fail(DG2P_EUNSUPPORTED, "the stream-function velocity is for the kinematic orders p = 1, 3");
  CurlArgs C{};
  const int n = m->desc.order + 1;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) C.D[a][b] = m->D[a][b];
  C.Jinv[0] = 1.0 / m->J[0];
  C.Jinv[1] = 1.0 / m->J[1];
  C.n = n;
  C.E = m->E;
  const long long total = m->E * m->nn;
  if (total == 0) return DG2P_OK;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_kin_curl, dim3((unsigned)((total + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, C, S, u0);
  return hip_check(hipGetLastError(), "kin_velocity_from_stream launch");
}

int dg2p_kin_max_dt(dg2p_mesh m, const dg2p_kin_params* kp, const double* u0, double cfl, double* dt, void* work,
                    void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !u0 || !dt) return fail(DG2P_EINVAL, "mesh, u0 and dt must be non-NULL");
  if (!(cfl > 0.0)) return fail(DG2P_EINVAL, "cfl must be > 0");
  int st = check_kin(m, kp);
  if (st) return st;
  st = check_ws(work, kin_work_bytes(m, DG2P_OP_KIN_AUX));
  if (st) return st;
  const KArgs A = kin_args(m, kp);
  hipStream_t s = (hipStream_t)stream;
  Work w;
  w.rec = static_cast<double*>(work);
  w.rec2 = w.rec + RATE * elem_blocks(m);
  long long nrec = elem_blocks(m);
  {
    TimedLaunch t(DG2P_K_RATE, s);
    if (m->desc.order == 1) {
      const long long n = m->E * m->nn;
      nrec = (n + BLOCK - 1) / BLOCK;
      const dim3 g((unsigned)nrec);
      if (m->dim == 1) hipLaunchKernelGGL(k_kin1_rate<1>, g, dim3(BLOCK), 0, s, n, u0, w.rec);
      else if (m->dim == 2) hipLaunchKernelGGL(k_kin1_rate<2>, g, dim3(BLOCK), 0, s, n, u0, w.rec);
      else hipLaunchKernelGGL(k_kin1_rate<3>, g, dim3(BLOCK), 0, s, n, u0, w.rec);
    } else if (m->dim == 1) {
      hipLaunchKernelGGL(k_kin_rate<1>, elem_grid(A), dim3(ewg<1>()), 0, s, A, u0, w.rec);
    } else if (m->dim == 2) {
      hipLaunchKernelGGL(k_kin_rate<2>, elem_grid(A), dim3(ewg<2>()), 0, s, A, u0, w.rec);
    } else {
      hipLaunchKernelGGL(k_kin_rate<3>, elem_grid(A), dim3(ewg<3>()), 0, s, A, u0, w.rec);
    }
  }
  finalize_rate(m, A, w, nrec, cfl, nullptr, dt, nullptr, s);
  return hip_check(hipGetLastError(), "kin_max_dt launch");
}

int dg2p_kin_errors(dg2p_mesh m, const double* phi, const double* phi0, double* out, void* work, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!m || !phi || !phi0 || !out) return fail(DG2P_EINVAL, "mesh, phi, phi0 and out must be non-NULL");
  int st = check_ws(work, kin_work_bytes(m, DG2P_OP_KIN_AUX));
  if (st) return st;
  dg2p_kin_params kp{1.0, 1.0, 1.0, 0.0, 0.0};
  const KArgs A = kin_args(m, &kp);
  hipStream_t s = (hipStream_t)stream;
  double* rec = static_cast<double*>(work);
  const long long nb = kin_err_blocks(m);
  const long long n = m->E * m->nn;
  if (m->desc.order == 1) {
    if (m->dim == 1) hipLaunchKernelGGL(k_kin1_errors<1>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, n, phi, phi0, rec);
    else if (m->dim == 2) hipLaunchKernelGGL(k_kin1_errors<2>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, n, phi, phi0, rec);
    else hipLaunchKernelGGL(k_kin1_errors<3>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, n, phi, phi0, rec);
  } else if (m->dim == 1) {
    hipLaunchKernelGGL(k_kin_errors<1>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, phi, phi0, rec);
  } else if (m->dim == 2) {
    hipLaunchKernelGGL(k_kin_errors<2>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, phi, phi0, rec);
  } else {
    hipLaunchKernelGGL(k_kin_errors<3>, dim3((unsigned)nb), dim3(BLOCK), 0, s, A, phi, phi0, rec);
  }
  hipLaunchKernelGGL(k_kin_sum, dim3(1), dim3(FIN_THREADS), 0, s, rec, nb, 3, out);
  return hip_check(hipGetLastError(), "kin_errors launch");
}

int dg2p_calibrate_fp64_fma(double* tflops, void* stream) {
  DG2P_API_RANGE();
  g_last_error.clear();
  if (!tflops) return fail(DG2P_EINVAL, "tflops must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(DG2P_EHIP, "hipEventCreate failed");
  }
  const dim3 grid(CALIB_WGS), block(CALIB_THREADS);
  double best_ms = 0.0;
  int st = DG2P_OK;
  for (int rep = 0; rep < 4 && st == DG2P_OK; ++rep) {
    (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_fma_calib, grid, block, 0, s, CALIB_ITERS, 1.0 - 1e-9, 1e-9, -1.0,
                       static_cast<double*>(nullptr));
    (void)hipEventRecord(e1, s);
    st = hip_check(hipEventSynchronize(e1), "fma calibration");
    float ms = 0.0f;
    if (st == DG2P_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && rep > 0 && (best_ms == 0.0 || ms < best_ms))
      best_ms = ms;  // the first launch warms the clocks up and is not counted
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DG2P_OK) return st;
  if (!(best_ms > 0.0)) return fail(DG2P_EHIP, "fma calibration: no elapsed time");
  const double flop = 2.0 * CALIB_CHAINS * (double)CALIB_ITERS * CALIB_WGS * CALIB_THREADS;
  *tflops = flop / (best_ms * 1e-3) / 1e12;
  return DG2P_OK;
}

int dg2p_timing_enable(int on) {
  if (on && !g_timing.created) {
    for (int i = 0; i < TIMING_SLOTS; ++i) {
      if (hipEventCreate(&g_timing.start[i]) != hipSuccess || hipEventCreate(&g_timing.stop[i]) != hipSuccess)
        return fail(DG2P_EHIP, "hipEventCreate failed");
    }
    g_timing.created = true;
  }
  g_timing.on = on != 0;
  if (on) g_timing.used = 0;
  return DG2P_OK;
}

int dg2p_timing_read(int kernel, double* mean_ms, long long* count) {
  if (!mean_ms || !count) return fail(DG2P_EINVAL, "mean_ms and count must be non-NULL");
  double sum = 0.0;
  long long n = 0;
  for (int i = 0; i < g_timing.used; ++i) {
    if (g_timing.kind[i] != kernel) continue;
    int st = hip_check(hipEventSynchronize(g_timing.stop[i]), "hipEventSynchronize");
    if (st) return st;
    float ms = 0.0f;
    st = hip_check(hipEventElapsedTime(&ms, g_timing.start[i], g_timing.stop[i]), "hipEventElapsedTime");
    if (st) return st;
    sum += ms;
    ++n;
  }
  *mean_ms = n ? sum / (double)n : 0.0;
  *count = n;
  return DG2P_OK;
}

}  // extern "C"
