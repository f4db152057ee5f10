// Stage and ingredient kernels of one (dimension, precision) pair.  Compiled
// once per pair with -DDG2P_DIM=d -DDG2P_PR=p (see the package's build step).

#include "dg2p_launch.hpp"

#ifndef DG2P_DIM
#error "DG2P_DIM must be defined (1, 2 or 3)"
#endif
#ifndef DG2P_PR
#error "DG2P_PR must be defined (0 FP64, 1 FP32, 2 BF16)"
#endif

namespace dg2p {

namespace {

template <int DIM, bool VISC, bool CSF, int BCK, int PR>
void stage_mode(int mode, int epi, const KArgs& A0, const StageIO& io, hipStream_t s) {
  const KArgs A = stage_args<DIM>(A0);
  const dim3 g((unsigned)(8 * A.xcd_chunk)), b(ewg<DIM>());
  if (mode == 0)
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 0, 0, PR>), g, b, 0, s, A, io);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 1, 1, PR>), g, b, 0, s, A, io);
  else if (epi == 1)
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 2, 1, PR>), g, b, 0, s, A, io);
  else if (epi == 2)
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 2, 2, PR>), g, b, 0, s, A, io);
  else if (epi == 3)
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 2, 3, PR>), g, b, 0, s, A, io);
  else
    hipLaunchKernelGGL((k_stage<DIM, VISC, CSF, BCK, 2, 0, PR>), g, b, 0, s, A, io);
}

template <int DIM, int BCK, int PR>
void stage_terms(bool visc, bool csf, int mode, int epi, const KArgs& A, const StageIO& io, hipStream_t s) {
  if (visc && csf) stage_mode<DIM, true, true, BCK, PR>(mode, epi, A, io, s);
  else if (visc) stage_mode<DIM, true, false, BCK, PR>(mode, epi, A, io, s);
  else if (csf) stage_mode<DIM, false, true, BCK, PR>(mode, epi, A, io, s);
  else stage_mode<DIM, false, false, BCK, PR>(mode, epi, A, io, s);
}

}  // namespace

template <int DIM, int PR>
void launch_stage_dp(int bck, bool visc, bool csf, int mode, int epi, const KArgs& A, const StageIO& io,
                     hipStream_t s) {
  if (bck == 2) stage_terms<DIM, 2, PR>(visc, csf, mode, epi, A, io, s);
  else if (bck == 1) stage_terms<DIM, 1, PR>(visc, csf, mode, epi, A, io, s);
  else stage_terms<DIM, 0, PR>(visc, csf, mode, epi, A, io, s);
}

template <int DIM, int PR>
void launch_ingredients_dp(bool visc, const KArgs& A, const double* U, double* G, double* rec, hipStream_t s) {
  const dim3 g((unsigned)(8 * A.xcd_chunk)), b(ewg<DIM>());
  if (visc) hipLaunchKernelGGL((k_ingredients<DIM, true, PR>), g, b, 0, s, A, U, G, rec);
  else hipLaunchKernelGGL((k_ingredients<DIM, false, PR>), g, b, 0, s, A, U, G, rec);
}

template void launch_stage_dp<DG2P_DIM, DG2P_PR>(int, bool, bool, int, int, const KArgs&, const StageIO&,
                                                 hipStream_t);
template void launch_ingredients_dp<DG2P_DIM, DG2P_PR>(bool, const KArgs&, const double*, double*, double*,
                                                       hipStream_t);

}  // namespace dg2p
