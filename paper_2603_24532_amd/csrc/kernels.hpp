// Host-side launchers of the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace mbpt {

size_t sample_lds_bytes(int nd, int nb, int block);
hipError_t launch_sample_single(const KArgs &a, int task, int order, int q, int prec, int nitems,
                                int block, hipStream_t st);
hipError_t launch_sample_batched(const KArgs &a, int q, int prec, int max_nd, int grid, int block,
                                 hipStream_t st);
hipError_t launch_finish(const KArgs &a, int first_task, int ntasks, int max_nd, double alpha,
                         hipStream_t st);
hipError_t launch_dump(const KArgs &a, int task, int order, int q, int prec, uint32_t iter,
                       uint64_t first, uint64_t count, double *out, hipStream_t st);
hipError_t launch_init(const KArgs &a, int first, int ntasks, hipStream_t st);
int batched_occupancy(int q, int prec, int max_nd, int block, size_t lds);

}  // namespace mbpt
