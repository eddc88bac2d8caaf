// Retrieval and deletion kernels for every (G, W).
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

hc_err launch_retrieve(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                       uint32_t* values_out, uint8_t* found_out, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_retrieve<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, n, values_out, found_out);
    return check_launch("retrieve");
  });
}

hc_err launch_erase(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                    uint8_t* status, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if (kind == KIND_MULTI) {
      auto k = k_erase<GG, WW, KIND_MULTI>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, n, status);
    } else {
      auto k = k_erase<GG, WW, KIND_SINGLE>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, t, work_for(n, GG, grid, stream), keys, n, status);
    }
    return check_launch("erase");
  });
}

}  // namespace hc
