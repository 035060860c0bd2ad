// Convolution-type transform kernels (RS column pass, vectorial mixing)
// for element type float, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_rs_cols<float>(int, cx<float>*, int64_t, int, int, const cx<float>*, int, bool, int,
                                       const cx<float>*, hipStream_t, int);
template hipError_t launch_mix2_cols<float>(int, const cx<float>*, const cx<float>*, cx<float>*, int64_t, int, int,
                                         const cx<float>*, int, float, const cx<float>*, int, float, bool, int, int,
                                         const cx<float>*, hipStream_t, int);
template int col_pass_lines<float>(int, int, int);
template int rs_cols_fill_variant<float>(int, int, int, int);
}  // namespace lp
