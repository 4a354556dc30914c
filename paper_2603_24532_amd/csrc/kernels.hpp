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
// The same items with a persistent grid (about as many blocks as are resident
// at once on `cus` compute units) claiming chunks of items from the order's
// counter a.queue[order] (zero at launch).
hipError_t launch_sample_persistent(const KArgs &a, int order, int q, int prec, bool group, int k0,
                                    int k1, int nitems, int block, int cus, hipStream_t st);
// Items of the tasks of the fourth-order diagram `id` (olist[k0, k1), nitems
// items from olist[k0].x) in nuclear matter with the quartic regulator and the
// polynomial label sums, fp64 (prec 0) or fp32 (1): the per-diagram kernel
// with compile-time descriptor masks (kernels_o4fixed.hip).
hipError_t launch_sample_order_fixed4(const KArgs &a, int id, int prec, int k0, int k1, int nitems,
                                      int block, hipStream_t st);
// Iteration end of tasks [first_task, first_task + ntasks) that take part in
// iteration step_iter of the current launch sequence (plan > step_iter).
hipError_t launch_finish(const KArgs &a, int first_task, int ntasks, int step_iter, double alpha,
                         hipStream_t st);
// out_reg (regularised components, count * nreg; may be null) is written only
// when a.nreg > 0.
hipError_t launch_dump(const KArgs &a, int task, int order, int q, int prec, bool group,
                       uint32_t iter, uint64_t first, uint64_t count, double *out, double *out_reg,
                       hipStream_t st);
// Zero histograms and running state of tasks [first, first + ntasks); grids
// to uniform and the Philox iteration word to 0 unless keep_grid.
hipError_t launch_init(const KArgs &a, int first, int ntasks, hipStream_t st,
                       bool keep_grid = false);
// HF spline tables of tasks [first, first + ntasks): ntab isospin tables each,
// partners summed over npartner isospins; gl = Gauss-Legendre (x, w) on the
// device.
hipError_t launch_hf(const KArgs &a, const double *gl, int first, int ntasks, int ntab,
                     int npartner, hipStream_t st);

// Per-(order, q) launchers, defined in kernels_inst.hip (one object per pair).
template <int ORDER, int Q>
hipError_t launch_single_oq(const KArgs &a, int t, int prec, bool group, int nitems, int block,
                            hipStream_t st);
template <int ORDER, int Q>
hipError_t launch_order_oq(const KArgs &a, int prec, bool group, int k0, int k1, int grid,
                           int block, hipStream_t st);
template <int ORDER, int Q>
hipError_t launch_persist_oq(const KArgs &a, int prec, bool group, int k0, int k1, int nitems,
                             int block, int cus, hipStream_t st);
template <int ORDER, int Q>
hipError_t launch_dump_oq(const KArgs &a, int t, int prec, bool group, uint32_t iter,
                          uint64_t first, uint64_t count, double *out, double *out_reg,
                          hipStream_t st);
// Per-diagram fourth-order launchers for the ids [FIRST, FIRST + kFixed4Chunk),
// one translation unit each.
constexpr int kFixed4Chunk = 10;
template <int FIRST>
hipError_t launch_o4_fixed(const KArgs &a, int id, int prec, int k0, int k1, int nitems, int block,
                           hipStream_t st);
template <>
hipError_t launch_o4_fixed<0>(const KArgs &, int, int, int, int, int, int, hipStream_t);
template <>
hipError_t launch_o4_fixed<10>(const KArgs &, int, int, int, int, int, int, hipStream_t);
template <>
hipError_t launch_o4_fixed<20>(const KArgs &, int, int, int, int, int, int, hipStream_t);
template <>
hipError_t launch_o4_fixed<30>(const KArgs &, int, int, int, int, int, int, hipStream_t);
#define MBPT_DECLARE_OQ(O, Q)                                                                   \
  template <>                                                                                   \
  hipError_t launch_single_oq<O, Q>(const KArgs &, int, int, bool, int, int, hipStream_t);      \
  template <>                                                                                   \
  hipError_t launch_order_oq<O, Q>(const KArgs &, int, bool, int, int, int, int, hipStream_t);  \
  template <>                                                                                   \
  hipError_t launch_persist_oq<O, Q>(const KArgs &, int, bool, int, int, int, int, int,         \
                                     hipStream_t);                                              \
  template <>                                                                                   \
  hipError_t launch_dump_oq<O, Q>(const KArgs &, int, int, bool, uint32_t, uint64_t, uint64_t,  \
                                  double *, double *, hipStream_t);
MBPT_DECLARE_OQ(1, 2)
MBPT_DECLARE_OQ(1, 4)
MBPT_DECLARE_OQ(2, 2)
MBPT_DECLARE_OQ(2, 4)
MBPT_DECLARE_OQ(3, 2)
MBPT_DECLARE_OQ(3, 4)
MBPT_DECLARE_OQ(4, 2)
MBPT_DECLARE_OQ(4, 4)
MBPT_DECLARE_OQ(5, 2)
MBPT_DECLARE_OQ(5, 4)
#undef MBPT_DECLARE_OQ

}  // namespace mbpt
