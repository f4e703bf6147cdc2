// Cluster kernels instantiated for double iterations, MODE_GIBBS.
#include "lrh_device.h"

namespace lrh {
template hipError_t launch_cluster_mode<double, false, MODE_GIBBS>(const ClusterArgs<double>&, int, int, hipStream_t);
template hipError_t launch_cluster_mode<double, true, MODE_GIBBS>(const ClusterArgs<double>&, int, int, hipStream_t);
}  // namespace lrh
