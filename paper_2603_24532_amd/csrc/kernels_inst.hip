// Sample, batched and per-sample-dump kernels of one order and matter,
// instantiated for every kernel mode, label-sum form and regulator-exponent
// class.  The build compiles this file once per (order, q) pair with
// -DMBPT_INST_ORDER=<1..5> -DMBPT_INST_Q=<2|4>, so the pairs build in
// parallel; kernels.hip dispatches to the launchers defined here.
#include "kernels_dev.hpp"

#include <algorithm>

#if !defined(MBPT_INST_ORDER) || !defined(MBPT_INST_Q)
#error "compile with -DMBPT_INST_ORDER=<order> -DMBPT_INST_Q=<2|4>"
#endif

namespace mbpt {
namespace {

constexpr int O = MBPT_INST_ORDER;
constexpr int Q = MBPT_INST_Q;

// Calls fn with the mode P (0..6) as a compile-time constant, the label-sum
// form X and the regulator-exponent class HE (2: quartic, fixed at compile
// time; 0: read at launch).
template <typename Fn>
hipError_t with_kernel(const KArgs &a, int m, Fn &&fn) {
  auto xh = [&](auto p) -> hipError_t {
    constexpr int P = decltype(p)::value;
    auto h = [&](auto x) -> hipError_t {
      constexpr bool X = decltype(x)::value;
      return a.phys.half_exp == 2 ? fn(std::integral_constant<int, P>{}, std::bool_constant<X>{},
                                       std::integral_constant<int, 2>{})
                                  : fn(std::integral_constant<int, P>{}, std::bool_constant<X>{},
                                       std::integral_constant<int, 0>{});
    };
    return a.label_mode ? h(std::true_type{}) : h(std::false_type{});
  };
  switch (m) {
    case 0: return xh(std::integral_constant<int, 0>{});
    case 1: return xh(std::integral_constant<int, 1>{});
    case 2: return xh(std::integral_constant<int, 2>{});
    case 3: return xh(std::integral_constant<int, 3>{});
    case 4: return xh(std::integral_constant<int, 4>{});
    case 5: return xh(std::integral_constant<int, 5>{});
    case 6: return xh(std::integral_constant<int, 6>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <>
hipError_t launch_single_oq<O, Q>(const KArgs &a, int t, int prec, bool group, int nitems,
                                  int block, hipStream_t st) {
  return with_kernel(a, mode_of(a, prec, group), [&](auto p, auto x, auto h) -> hipError_t {
    constexpr int P = decltype(p)::value;
    constexpr bool X = decltype(x)::value;
    constexpr int HE = decltype(h)::value;
    const size_t lds = sample_lds_bytes(3 * (O + 1), a.phys.nb, block, lds_tables<Q, P>()) +
                       cycle_lds_bytes<O, Q, P, X>();
    hipLaunchKernelGGL((sample_single<O, Q, P, X, HE>), dim3(nitems), dim3(block), lds, st, a, t);
    return hipGetLastError();
  });
}

template <>
hipError_t launch_order_oq<O, Q>(const KArgs &a, int prec, bool group, int k0, int k1, int grid,
                                 int block, hipStream_t st) {
  return with_kernel(a, mode_of(a, prec, group), [&](auto p, auto x, auto h) -> hipError_t {
    constexpr int P = decltype(p)::value;
    constexpr bool X = decltype(x)::value;
    constexpr int HE = decltype(h)::value;
    const size_t lds = sample_lds_bytes(3 * (O + 1), a.phys.nb, block, lds_tables<Q, P>()) +
                       cycle_lds_bytes<O, Q, P, X>();
    hipLaunchKernelGGL((sample_order<O, Q, P, X, HE>), dim3(grid), dim3(block), lds, st, a, k0,
                       k1);
    return hipGetLastError();
  });
}

template <>
hipError_t launch_persist_oq<O, Q>(const KArgs &a, int prec, bool group, int k0, int k1, int nitems,
                                   int block, int cus, hipStream_t st) {
  if (!a.queue) return hipErrorInvalidValue;
  return with_kernel(a, mode_of(a, prec, group), [&](auto p, auto x, auto h) -> hipError_t {
    constexpr int P = decltype(p)::value;
    constexpr bool X = decltype(x)::value;
    constexpr int HE = decltype(h)::value;
    const size_t lds = sample_lds_bytes(3 * (O + 1), a.phys.nb, block, lds_tables<Q, P>()) +
                       cycle_lds_bytes<O, Q, P, X>();
    auto kern = sample_persistent<O, Q, P, X, HE>;
    // more blocks than can be resident: the extra ones start as others
    // finish and find the counter exhausted, so the device stays full
    // whatever the occupancy of this kernel
    const int grid = std::max(1, std::min(nitems, kPersistentBlocksPerCu * std::max(1, cus)));
    // about eight claims per block: small enough chunks to balance the
    // blocks' finishing times, large enough to keep a block on one task
    const int chunk = std::max(1, nitems / (8 * grid));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, a, k0, k1, nitems, chunk);
    return hipGetLastError();
  });
}

// The dump kernels take the same exponent class as the sample kernels, so
// dumped weights come from the arithmetic the integration runs.
template <>
hipError_t launch_dump_oq<O, Q>(const KArgs &a, int t, int prec, bool group, uint32_t iter,
                                uint64_t first, uint64_t count, double *out, double *out_reg,
                                hipStream_t st) {
  return with_kernel(a, mode_of(a, prec, group), [&](auto p, auto x, auto h) -> hipError_t {
    constexpr int P = decltype(p)::value;
    constexpr bool X = decltype(x)::value;
    constexpr int HE = decltype(h)::value;
    const int block = 256;
    const dim3 grid(static_cast<unsigned>((count + block - 1) / block));
    const size_t lds = fixed_lds_bytes() + hf_lds_doubles(lds_tables<Q, P>()) * sizeof(double) +
                       2 * static_cast<size_t>(3 * (O + 1)) * a.phys.nb * sizeof(double) +
                       cycle_lds_bytes<O, Q, P, X>();
    hipLaunchKernelGGL((dump_samples<O, Q, P, X, HE>), grid, dim3(block), lds, st, a, t, iter,
                       first, count, out, out_reg);
    return hipGetLastError();
  });
}

}  // namespace mbpt
