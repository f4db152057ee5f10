// Residual VJP kernels of one dimension.  Compiled once per dimension with
// -DDG2P_DIM=d (see the package's build step).

#include "dg2p_adjoint.hpp"
#include "dg2p_launch.hpp"

#ifndef DG2P_DIM
#error "DG2P_DIM must be defined (1, 2 or 3)"
#endif

namespace dg2p {

namespace {

template <int DIM, bool VISC, bool CSF, bool WALLS>
void vjp_passes(const KArgs& A, const VjpIO& io, hipStream_t s) {
  const dim3 g((unsigned)(8 * A.xcd_chunk)), b(ewg<DIM>());
  hipLaunchKernelGGL((k_vjp_local<DIM, VISC, CSF, WALLS>), g, b, 0, s, A, io);
  hipLaunchKernelGGL((k_vjp_gather<DIM, VISC, WALLS>), g, b, 0, s, A, io);
}
template <int DIM, bool WALLS>
void vjp_kinds(bool visc, bool csf, const KArgs& A, const VjpIO& io, hipStream_t s) {
  if (visc && csf) vjp_passes<DIM, true, true, WALLS>(A, io, s);
  else if (visc) vjp_passes<DIM, true, false, WALLS>(A, io, s);
  else if (csf) vjp_passes<DIM, false, true, WALLS>(A, io, s);
  else vjp_passes<DIM, false, false, WALLS>(A, io, s);
}

}  // namespace

template <int DIM>
void launch_vjp_dim(bool visc, bool csf, bool walls, const KArgs& A, const VjpIO& io, hipStream_t s) {
  if (walls) vjp_kinds<DIM, true>(visc, csf, A, io, s);
  else vjp_kinds<DIM, false>(visc, csf, A, io, s);
}

template void launch_vjp_dim<DG2P_DIM>(bool, bool, bool, const KArgs&, const VjpIO&, hipStream_t);

}  // namespace dg2p
