// Cluster kernels instantiated for float iterations, MODE_GROUND.
#include "lrh_device.h"

namespace lrh {
template hipError_t launch_cluster_mode<float, false, MODE_GROUND>(const ClusterArgs<float>&, int, int, hipStream_t);
template hipError_t launch_cluster_mode<float, true, MODE_GROUND>(const ClusterArgs<float>&, int, int, hipStream_t);
}  // namespace lrh
