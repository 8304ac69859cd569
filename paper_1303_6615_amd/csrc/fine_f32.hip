// Fine-batch kernels, FP32 propagators: every workgroup shape of every grid size.
#include "dispatch.hpp"
#include "fine_kernel.hpp"
#include "launch.hpp"

namespace ap {

hipError_t launch_fine_f32(int nx, int shape, const cx<double>* in, cx<double>* out, int batch, int steps,
                           const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s) {
  AP_DISPATCH_NX(nx, (fine_launch_config<float, NX>(shape, in, out, batch, steps, coef64, coef32, t, s)));
}
int fine_shape_f32(int nx, int shape, int* slices) {
  AP_DISPATCH_NX_INT(nx, (fine_shape_info<float, NX>(shape, slices)));
}

}  // namespace ap
