// Convolution-type transform kernels (RS column pass, vectorial mixing)
// for element type double, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_rs_cols<double>(int, cx<double>*, int64_t, int, int, const cx<double>*, int, bool, int,
                                       const cx<double>*, hipStream_t, int);
template hipError_t launch_mix2_cols<double>(int, const cx<double>*, const cx<double>*, cx<double>*, int64_t, int, int,
                                         const cx<double>*, int, double, const cx<double>*, int, double, bool, int, int,
                                         const cx<double>*, hipStream_t, int);
template int col_pass_lines<double>(int, int, int);
template int rs_cols_fill_variant<double>(int, int, int, int);
}  // namespace lp
