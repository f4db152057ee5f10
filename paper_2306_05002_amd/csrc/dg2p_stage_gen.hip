// Stage, ingredient and record kernels of quadrilaterals of degree != 3
// (p = 4), FP64.

#include "dg2p_launch.hpp"
#include "dg2p_stage_gen.hpp"

namespace dg2p {

namespace {

constexpr int GEN_P = 4;

template <bool VISC, bool CSF, int BCK>
void gen_stage(int mode, int epi, const KArgs& A, const StageIO& io, hipStream_t s) {
  const dim3 g((unsigned)(8 * A.xcd_chunk)), b(64);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 0, 0>), g, b, 0, s, A, io);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 1, 1>), g, b, 0, s, A, io);
  else if (epi == 1)
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 2, 1>), g, b, 0, s, A, io);
  else if (epi == 2)
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 2, 2>), g, b, 0, s, A, io);
  else if (epi == 3)
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 2, 3>), g, b, 0, s, A, io);
  else
    hipLaunchKernelGGL((k_stage_g<GEN_P, VISC, CSF, BCK, 2, 0>), g, b, 0, s, A, io);
}

template <int BCK>
void gen_terms(bool visc, bool csf, int mode, int epi, const KArgs& A, const StageIO& io, hipStream_t s) {
  if (visc && csf) gen_stage<true, true, BCK>(mode, epi, A, io, s);
  else if (visc) gen_stage<true, false, BCK>(mode, epi, A, io, s);
  else if (csf) gen_stage<false, true, BCK>(mode, epi, A, io, s);
  else gen_stage<false, false, BCK>(mode, epi, A, io, s);
}

}  // namespace

// Only p = 4 is instantiated; the host admits no other generic order.
void launch_stage_gen(int order, int bck, bool visc, bool csf, int mode, int epi, const KArgs& A,
                      const StageIO& io, hipStream_t s) {
  (void)order;
  if (bck == 2) gen_terms<2>(visc, csf, mode, epi, A, io, s);
  else if (bck == 1) gen_terms<1>(visc, csf, mode, epi, A, io, s);
  else gen_terms<0>(visc, csf, mode, epi, A, io, s);
}

void launch_ingredients_gen(int order, bool visc, const KArgs& A, const double* U, double* G, double* rec,
                            hipStream_t s) {
  (void)order;
  const dim3 g((unsigned)(8 * A.xcd_chunk)), b(64);
  if (visc) hipLaunchKernelGGL((k_ingredients_g<GEN_P, true>), g, b, 0, s, A, U, G, rec);
  else hipLaunchKernelGGL((k_ingredients_g<GEN_P, false>), g, b, 0, s, A, U, G, rec);
}

void launch_records_gen(int order, bool visc, unsigned blocks, const KArgs& A, const double* U, double* rec,
                        hipStream_t s) {
  (void)order;
  if (visc) hipLaunchKernelGGL((k_records_g<GEN_P, true>), dim3(blocks), dim3(BLOCK), 0, s, A, U, rec);
  else hipLaunchKernelGGL((k_records_g<GEN_P, false>), dim3(blocks), dim3(BLOCK), 0, s, A, U, rec);
}

}  // namespace dg2p
