// Launchers of the element-pass kernels, one set per (dimension, precision).
//
// Each set is defined in its own translation unit (dg2p_stage_inst.hip,
// compiled once per DIM and PR; dg2p_vjp_inst.hip, once per DIM), so the
// stage-kernel variants of the library compile in parallel.  The host entry
// points in dg2p.hip see only these declarations.

#pragma once

#include <hip/hip_runtime.h>

#include "dg2p_device.hpp"

namespace dg2p {

struct VjpIO;

// Stage pass (k_stage) of dimension DIM and contraction precision PR with the
// boundary class bck (0 periodic, 1 walls / extrapolation, 2 also Dirichlet /
// Riemann), viscous and CSF terms on or off, MODE 0 (store R), 1 (first
// stage) or 2 (later stages), and epilogue epi (0 none, 1 face ingredients,
// 2 ingredients + monitor records, 3 ingredients + rate records).
template <int DIM, int PR>
void launch_stage_dp(int bck, bool visc, bool csf, int mode, int epi, const KArgs& A, const StageIO& io,
                     hipStream_t s);

// Ingredient pass (k_ingredients): face ingredients and rate records of U.
template <int DIM, int PR>
void launch_ingredients_dp(bool visc, const KArgs& A, const double* U, double* G, double* rec, hipStream_t s);

// Quadrilaterals of degree `order` != 3 (dg2p_stage_gen.hip): stage pass,
// ingredient pass and standalone records (grid of `blocks` workgroups).
void launch_stage_gen(int order, int bck, bool visc, bool csf, int mode, int epi, const KArgs& A,
                      const StageIO& io, hipStream_t s);
void launch_ingredients_gen(int order, bool visc, const KArgs& A, const double* U, double* G, double* rec,
                            hipStream_t s);
void launch_records_gen(int order, bool visc, unsigned blocks, const KArgs& A, const double* U, double* rec,
                        hipStream_t s);

// Residual VJP passes (k_vjp_local, k_vjp_gather) of dimension DIM.
template <int DIM>
void launch_vjp_dim(bool visc, bool csf, bool walls, const KArgs& A, const VjpIO& io, hipStream_t s);

}  // namespace dg2p
