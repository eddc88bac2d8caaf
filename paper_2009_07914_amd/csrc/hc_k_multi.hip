// Multi-value count and write kernels for every (G, W).
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

hc_err launch_count_multi(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                          uint32_t* counts, uint64_t* offsets, uint8_t* found_out, uint32_t budget,
                          uint64_t* long_list, unsigned long long* long_n, uint64_t long_cap, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_count_multi<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, n, counts, offsets,
                       found_out, budget, long_list, long_n, long_cap);
    return check_launch("count_values");
  });
}

hc_err launch_write_multi(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                          const uint64_t* offsets, uint32_t* out, uint32_t budget, uint64_t* long_list,
                          unsigned long long* long_n, uint64_t long_cap, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_write_multi<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, n, offsets, out, budget,
                       long_list, long_n, long_cap);
    return check_launch("retrieve_all");
  });
}

}  // namespace hc
