// Per-diagram fourth-order nuclear-matter sample kernels (compile-time
// descriptor masks, quartic regulator, polynomial label sums, fp64 and fp32)
// for the diagram ids [MBPT_FIXED_FIRST, MBPT_FIXED_FIRST + MBPT_FIXED_COUNT):
// the build compiles the 39 ids in a few units in parallel.
#include "kernels_dev.hpp"

#include <utility>

#if !defined(MBPT_FIXED_FIRST) || !defined(MBPT_FIXED_COUNT)
#error "compile with -DMBPT_FIXED_FIRST=<first id> -DMBPT_FIXED_COUNT=<ids>"
#endif

namespace mbpt {
namespace {

template <int V>
hipError_t launch_one(const KArgs &a, int prec, int k0, int k1, int nitems, int block,
                      hipStream_t st) {
  constexpr int O = 4, Q = 4;
  auto go = [&](auto p) -> hipError_t {
    constexpr int P = decltype(p)::value;
    const size_t lds = sample_lds_bytes(3 * (O + 1), a.phys.nb, block, lds_tables<Q, P>()) +
                       cycle_lds_bytes<O, Q, P, false>();
    hipLaunchKernelGGL((sample_order_fixed<O, Q, P, 2, V>), dim3(nitems), dim3(block), lds, st, a,
                       k0, k1);
    return hipGetLastError();
  };
  return prec ? go(std::integral_constant<int, 1>{}) : go(std::integral_constant<int, 0>{});
}

template <int... I>
hipError_t dispatch(std::integer_sequence<int, I...>, int id, const KArgs &a, int prec, int k0,
                    int k1, int nitems, int block, hipStream_t st) {
  hipError_t r = hipErrorInvalidValue;
  (void)((id == MBPT_FIXED_FIRST + I
              ? (r = launch_one<MBPT_FIXED_FIRST + I>(a, prec, k0, k1, nitems, block, st), true)
              : false) ||
         ...);
  return r;
}

}  // namespace

template <>
hipError_t launch_o4_fixed<MBPT_FIXED_FIRST>(const KArgs &a, int id, int prec, int k0, int k1,
                                             int nitems, int block, hipStream_t st) {
  return dispatch(std::make_integer_sequence<int, MBPT_FIXED_COUNT>{}, id, a, prec, k0, k1,
                  nitems, block, st);
}

}  // namespace mbpt
