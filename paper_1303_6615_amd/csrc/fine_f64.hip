// Fine-batch kernels, all FP64: every workgroup shape of every grid size.
#include "dispatch.hpp"
#include "fine_kernel.hpp"
#include "launch.hpp"

namespace ap {

hipError_t launch_fine_f64(int nx, int shape, const cx<double>* in, cx<double>* out, int batch, int steps,
                           const cx<double>* coef64, const DevTables& t, hipStream_t s) {
  AP_DISPATCH_NX(nx, (fine_launch_config<double, NX>(shape, in, out, batch, steps, coef64, coef64, t, s)));
}
int fine_shape_f64(int nx, int shape, int* slices) {
  AP_DISPATCH_NX_INT(nx, (fine_shape_info<double, NX>(shape, slices)));
}

}  // namespace ap
