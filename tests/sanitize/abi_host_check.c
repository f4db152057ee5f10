/* Host-side exercise of libdg2p's C ABI for a build whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer: every entry point's
 * argument, descriptor, parameter and workspace checks, mesh creation for
 * every dimension, order and boundary kind, the host-side layout queries and
 * workspace arithmetic.  No call reaches the GPU (each one returns before its
 * first HIP call), so it runs without one.  Prints each mismatch of a status
 * code and exits 1 if there was any; a sanitizer report aborts the process. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/dg2p.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    fprintf(stderr, "MISMATCH %s: status %d, expected %d (%s)\n", what, got, want, dg2p_last_error());
    ++failures;
  }
}

static dg2p_mesh_desc box(int dim, int order, int n) {
  dg2p_mesh_desc d;
  memset(&d, 0, sizeof d);
  d.dim = dim;
  d.order = order;
  for (int k = 0; k < 3; ++k) {
    d.n_elem[k] = n + k;
    d.lo[k] = -0.5;
    d.hi[k] = 0.5 + 0.25 * k;
  }
  return d;
}

static dg2p_params params(int visc, double sigma, int precision) {
  dg2p_params p;
  memset(&p, 0, sizeof p);
  p.gamma[0] = 1.4;
  p.gamma[1] = 4.4;
  p.pinf[1] = 6000.0;
  p.rho0[0] = 1e-3;
  p.rho0[1] = 1.0;
  p.Gamma = 1.0;
  p.eps = 0.01;
  p.mu[0] = visc ? 1e-3 : 0.0;
  p.mu[1] = visc ? 1e-2 : 0.0;
  p.sigma = sigma;
  p.g[1] = -1.0;
  p.c_ip = 1.0;
  p.grad_reg = 1e-12;
  p.precision = precision;
  return p;
}

int main(void) {
  /* strings */
  if (!strstr(dg2p_version(), "gfx950")) ++failures;
  for (int s = -8; s <= 2; ++s)
    if (!dg2p_status_string(s)) ++failures;
  (void)dg2p_last_error();

  /* descriptors: every dimension, order and boundary kind */
  static const int orders[3] = {1, 3, 4};
  for (int dim = 1; dim <= 3; ++dim)
    for (int oi = 0; oi < 3; ++oi)
      for (int kind = DG2P_BC_PERIODIC; kind <= DG2P_BC_RIEMANN; ++kind) {
        dg2p_mesh_desc d = box(dim, orders[oi], 3);
        for (int k = 0; k < 3; ++k) {
          d.bc[k][0] = d.bc[k][1] = kind;
          d.bc_state[k][0][0] = d.bc_state[k][1][0] = 1.0;
        }
        dg2p_mesh m = NULL;
        const int want = (orders[oi] == 4 && dim != 2) ? DG2P_EUNSUPPORTED : DG2P_OK;
        expect(dg2p_create_mesh(&d, &m), want, "create_mesh");
        if (!m) continue;
        int nf = 0, nn = 0;
        long long E = 0;
        expect(dg2p_layout(m, &nf, &E, &nn), DG2P_OK, "layout");
        double* xyz = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)E * (size_t)nn);
        double* W = (double*)malloc(sizeof(double) * (size_t)nn);
        expect(dg2p_node_coords(m, xyz), DG2P_OK, "node_coords");
        expect(dg2p_node_weights(m, W), DG2P_OK, "node_weights");
        free(xyz);
        free(W);
        for (int visc = 0; visc < 2; ++visc)
          for (int prec = DG2P_FP64; prec <= DG2P_MIXED_BF16; ++prec) {
            dg2p_params p = params(visc, visc ? 0.07 : 0.0, prec);
            for (int op = DG2P_OP_RHS; op <= DG2P_OP_ADVANCE; ++op) {
              size_t bytes = 0;
              (void)dg2p_workspace_size(m, &p, op, &bytes);
            }
          }
        for (int op = DG2P_OP_KIN_RHS; op <= DG2P_OP_KIN_AUX; ++op) {
          size_t bytes = 0;
          (void)dg2p_kin_workspace_size(m, op, &bytes);
        }
        double nu = 0.0, dtau = 0.0;
        (void)dg2p_kin_reinit_params(m, 0.1, &nu, &dtau);
        /* hot entry points: every one rejects a missing workspace or a NULL
           array before launching anything (the device pointers are never
           dereferenced on the host) */
        dg2p_params p = params(1, 0.07, DG2P_FP64);
        double* fake = (double*)(size_t)0x1000;
        double R_dummy = 0.0;
        (void)R_dummy;
        if (orders[oi] != 1) {
          expect(dg2p_rhs(m, &p, fake, fake + 64, NULL, NULL), DG2P_EWORKSPACE, "rhs without workspace");
          expect(dg2p_rk_step(m, &p, fake, fake + 64, NULL, NULL), DG2P_EWORKSPACE, "rk_step without workspace");
          expect(dg2p_max_dt(m, &p, fake, 0.1, fake + 64, NULL, NULL, NULL), DG2P_EWORKSPACE,
                 "max_dt without workspace");
          expect(dg2p_advance(m, &p, fake, 1, 0.1, NULL, NULL, NULL, NULL, 0.0, NULL, NULL, NULL),
                 DG2P_EWORKSPACE, "advance without workspace");
        }
        expect(dg2p_rhs(m, &p, NULL, fake, NULL, NULL), DG2P_EINVAL, "rhs NULL U");
        expect(dg2p_rhs(m, NULL, fake, fake + 64, NULL, NULL), DG2P_EINVAL, "rhs NULL params");
        expect(dg2p_rk_step_noalloc(m, &p, NULL, fake, NULL), DG2P_EINVAL, "rk_step_noalloc NULL U");
        expect(dg2p_advance_monitored(m, &p, fake, 1, 0.1, NULL, NULL, NULL, NULL, 0.0, NULL, NULL, NULL),
               DG2P_EINVAL, "advance_monitored NULL monitors");
        expect(dg2p_destroy_mesh(m), DG2P_OK, "destroy_mesh");
      }

  /* bad descriptors */
  {
    dg2p_mesh m = NULL;
    dg2p_mesh_desc d = box(2, 3, 4);
    expect(dg2p_create_mesh(NULL, &m), DG2P_EINVAL, "create_mesh NULL desc");
    d.dim = 4;
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "dim 4");
    d = box(2, 2, 4);
    expect(dg2p_create_mesh(&d, &m), DG2P_EUNSUPPORTED, "order 2");
    d = box(2, 3, 4);
    d.n_elem[1] = 0;
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "no elements");
    d = box(3, 3, 4);
    d.n_elem[0] = d.n_elem[1] = d.n_elem[2] = 2147483647; /* product beyond 64 bits */
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "huge element counts");
    d = box(2, 3, 4);
    d.hi[0] = d.lo[0];
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "empty box");
    d = box(2, 3, 4);
    d.bc[0][0] = 9;
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "unknown boundary kind");
    d = box(2, 3, 4);
    d.bc[1][1] = DG2P_BC_SLIP_WALL;
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "periodic on one side");
    d = box(2, 3, 4);
    d.bc[1][0] = DG2P_BC_SLIP_WALL;
    d.bc[1][1] = DG2P_BC_RIEMANN;
    expect(dg2p_create_mesh(&d, &m), DG2P_EINVAL, "Riemann without pressure");
    if (m) ++failures;
  }

  /* bad parameters, on a valid mesh */
  {
    dg2p_mesh m = NULL;
    dg2p_mesh_desc d = box(2, 3, 4);
    expect(dg2p_create_mesh(&d, &m), DG2P_OK, "create_mesh");
    size_t bytes = 0;
    dg2p_params p = params(1, 0.07, DG2P_FP64);
    expect(dg2p_workspace_size(m, &p, DG2P_OP_ADVANCE, &bytes), DG2P_OK, "workspace_size");
    if (bytes == 0) ++failures;
    expect(dg2p_workspace_size(m, &p, 99, &bytes), DG2P_EINVAL, "unknown op");
    expect(dg2p_workspace_size(m, &p, DG2P_OP_RHS, NULL), DG2P_EINVAL, "workspace_size NULL out");
    p.gamma[0] = 1.0;
    expect(dg2p_workspace_size(m, &p, DG2P_OP_RHS, &bytes), DG2P_EINVAL, "gamma 1");
    p = params(1, 0.07, DG2P_FP64);
    p.eps = 0.0;
    expect(dg2p_workspace_size(m, &p, DG2P_OP_RHS, &bytes), DG2P_EINVAL, "eps 0");
    p = params(1, 0.07, 7);
    expect(dg2p_workspace_size(m, &p, DG2P_OP_RHS, &bytes), DG2P_EINVAL, "unknown precision");
    p = params(1, 0.07, DG2P_FP64);
    p.mu[1] = -1.0;
    expect(dg2p_workspace_size(m, &p, DG2P_OP_RHS, &bytes), DG2P_EINVAL, "negative viscosity");
    expect(dg2p_destroy_mesh(m), DG2P_OK, "destroy_mesh");
  }

  /* utilities that reject their arguments before any device call */
  expect(dg2p_calibrate_fp64_fma(NULL, NULL), DG2P_EINVAL, "calibrate NULL");
  expect(dg2p_timing_read(0, NULL, NULL), DG2P_EINVAL, "timing_read NULL");
  expect(dg2p_timing_enable(0), DG2P_OK, "timing_enable(0)");
  expect(dg2p_destroy_mesh(NULL), DG2P_OK, "destroy_mesh NULL");
  if (dg2p_noalloc_scratch_bytes() == 0) ++failures;

  if (failures) {
    fprintf(stderr, "%d mismatches\n", failures);
    return 1;
  }
  printf("abi host check: all statuses as expected\n");
  return 0;
}
