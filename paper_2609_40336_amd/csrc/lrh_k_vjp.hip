// Adjoint (Daleckii-Krein VJP) cluster kernels: launcher and instantiations.
#include "lrh_device.h"

namespace lrh {

hipError_t launch_cluster_vjp(const ClusterArgs<double>& a, bool cplx, int mode, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 g((unsigned)a.n), b(64);
#define VJP_CASE(DE)                                                                                   \
  if (a.De == DE) {                                                                                    \
    if (mode == MODE_GIBBS) {                                                                          \
      if (cplx) hipLaunchKernelGGL((k_cluster_vjp<double, true, DE, MODE_GIBBS>), g, b, 0, s, a);      \
      else hipLaunchKernelGGL((k_cluster_vjp<double, false, DE, MODE_GIBBS>), g, b, 0, s, a);          \
    } else {                                                                                           \
      if (cplx) hipLaunchKernelGGL((k_cluster_vjp<double, true, DE, MODE_GROUND>), g, b, 0, s, a);     \
      else hipLaunchKernelGGL((k_cluster_vjp<double, false, DE, MODE_GROUND>), g, b, 0, s, a);         \
    }                                                                                                  \
    return hipGetLastError();                                                                          \
  }
  VJP_CASE(2)
  VJP_CASE(4)
  VJP_CASE(8)
  VJP_CASE(16)
  VJP_CASE(32)
  if (a.De == 64 && !cplx) {
    if (mode == MODE_GIBBS) hipLaunchKernelGGL((k_cluster_vjp<double, false, 64, MODE_GIBBS>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_cluster_vjp<double, false, 64, MODE_GROUND>), g, b, 0, s, a);
    return hipGetLastError();
  }
#undef VJP_CASE
  return hipErrorInvalidValue;
}

}  // namespace lrh
