// Pipelined solve kernels, FP64: one grid size per launch.
#include "pipeline.hpp"

namespace ap {

hipError_t pipe_launch_f64(int nx, size_t lds, const PipeJob* jobs, int njobs, const void* probs,
                             int* ticket, int* abort, int* progress, unsigned long long* trace, int grid,
                             hipStream_t s) {
  AP_DISPATCH_NX(nx, (pipeline_launch<double, NX>(lds, jobs, njobs, probs, ticket, abort, progress, trace, grid, s)));
}
int pipe_occupancy_f64(int nx, size_t lds) {
  AP_DISPATCH_NX_INT(nx, (pipeline_occupancy<double, NX>(lds)));
}

}  // namespace ap
