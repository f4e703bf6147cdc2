// Cluster kernels instantiated for double iterations, MODE_GROUND.
#include "lrh_device.h"

namespace lrh {
template hipError_t launch_cluster_mode<double, false, MODE_GROUND>(const ClusterArgs<double>&, int, int, hipStream_t);
template hipError_t launch_cluster_mode<double, true, MODE_GROUND>(const ClusterArgs<double>&, int, int, hipStream_t);
}  // namespace lrh
