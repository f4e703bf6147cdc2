// Cluster kernels instantiated for double iterations, MODE_CERTIFY.
#include "lrh_device.h"

namespace lrh {
template hipError_t launch_cluster_mode<double, false, MODE_CERTIFY>(const ClusterArgs<double>&, int, int, hipStream_t);
template hipError_t launch_cluster_mode<double, true, MODE_CERTIFY>(const ClusterArgs<double>&, int, int, hipStream_t);
}  // namespace lrh
