// Launchers of the lane kernel (one LP per lane, simplex_lane.hpp), in a
// translation unit of their own that compiles beside the register-tile
// kernels.  The variant table (variants.hpp) names the instantiations.
#include "aux_kernels.hpp"
#include "blp_kernels.hpp"
#include "simplex_common.hpp"
#include "simplex_lane.hpp"
#include "variants.hpp"

namespace blp {

template <int R, int C, int NWV, int WPE>
hipError_t launch_lane(const KParams& P, int grid, hipStream_t s) {
    hipLaunchKernelGGL((simplex_lane_kernel<R, C, NWV, WPE>), dim3(grid), dim3(NWV * 64), 0, s, P);
    return hipGetLastError();
}
template <int R, int C, int NWV, int WPE>
const void* kernel_ptr_lane() {
    return reinterpret_cast<const void*>(&simplex_lane_kernel<R, C, NWV, WPE>);
}

// the lane variants of the table, and nothing else
#define BLP_LANE_VARIANT(NAME, R, C, NWV, WPE)                                        \
    template hipError_t launch_lane<R, C, NWV, WPE>(const KParams&, int, hipStream_t); \
    template const void* kernel_ptr_lane<R, C, NWV, WPE>();
#define BLP_REG_VARIANT(...)
#define BLP_BLK_VARIANT(...)
#define BLP_COLS_VARIANT(...)
BLP_REG_VARIANT_LIST

}  // namespace blp
