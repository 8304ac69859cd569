// Pipelined solve kernels, FP32: problems of grid sizes 64, 128, 256, 512, 1024, 2048 in one launch.
#include "pipeline.hpp"

namespace ap {

hipError_t pipe_launch_mix2048_f32(int, size_t lds, const PipeJob* jobs, int njobs, const void* probs,
                             int* ticket, int* abort, int* progress, unsigned long long* trace, int grid,
                             hipStream_t s) {
  return pipeline_launch<float, 64, 128, 256, 512, 1024, 2048>(lds, jobs, njobs, probs, ticket, abort, progress, trace, grid, s);
}
int pipe_occupancy_mix2048_f32(int, size_t lds) { return pipeline_occupancy<float, 64, 128, 256, 512, 1024, 2048>(lds); }

}  // namespace ap
