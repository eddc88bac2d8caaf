// Insert kernels (single-value, counting, multi-value) for every (G, W).
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

hc_err launch_insert(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys,
                     const uint32_t* values, uint64_t n, uint8_t* status, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if (kind == KIND_SINGLE) {
      auto k = k_insert_unique<GG, WW, KIND_SINGLE>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, values, n, status);
    } else if (kind == KIND_COUNT) {
      return launch_count_insert(t, GG, WW, keys, n, status, stream);
    } else {
      auto k = k_insert_multi<GG, WW>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, values, n, status);
    }
    return check_launch("insert");
  });
}

}  // namespace hc
