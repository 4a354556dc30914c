// Host-side launchers of the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace mbpt {

// Dynamic LDS of a sample kernel; ntab = HF spline tables held (0, 1 or 2).
size_t sample_lds_bytes(int nd, int nb, int block, int ntab);
// group: tasks of several descriptors may be present (diagram groups).
hipError_t launch_sample_single(const KArgs &a, int task, int order, int q, int prec, bool group,
                                int nitems, int block, hipStream_t st);
// Items [olist[k0].x, olist[k0].x + nitems) of the tasks listed in olist[k0, k1).
hipError_t launch_sample_order(const KArgs &a, int order, int q, int prec, bool group, int k0,
                               int k1, int nitems, int block, hipStream_t st);
// Iteration end of tasks [first_task, first_task + ntasks) that take part in
// iteration step_iter of the current launch sequence (plan > step_iter).
hipError_t launch_finish(const KArgs &a, int first_task, int ntasks, int step_iter, double alpha,
                         hipStream_t st);
// out_reg (regularised components, count * nreg; may be null) is written only
// when a.nreg > 0.
hipError_t launch_dump(const KArgs &a, int task, int order, int q, int prec, bool group,
                       uint32_t iter, uint64_t first, uint64_t count, double *out, double *out_reg,
                       hipStream_t st);
hipError_t launch_init(const KArgs &a, int first, int ntasks, hipStream_t st);
// HF spline tables of tasks [first, first + ntasks): ntab isospin tables each,
// partners summed over npartner isospins; gl = Gauss-Legendre (x, w) on the
// device.
hipError_t launch_hf(const KArgs &a, const double *gl, int first, int ntasks, int ntab,
                     int npartner, hipStream_t st);

}  // namespace mbpt
