// Convolution-type transform kernels (RS column pass, vectorial mixing,
// Bluestein) for element type double, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_rs_cols<double>(int, cx<double>*, int64_t, int, int, const cx<double>*, int, bool, int,
                                       const cx<double>*, hipStream_t, int);
template hipError_t launch_mix2_cols<double>(int, const cx<double>*, const cx<double>*, cx<double>*, int64_t, int, int,
                                         const cx<double>*, int, double, const cx<double>*, int, double, bool, int, int,
                                         const cx<double>*, hipStream_t, int);
template hipError_t launch_bluestein<double>(int, bool, const cx<double>*, cx<double>*, Lines, Lines, int, int, int,
                                         const cx<double>*, const cx<double>*, const cx<double>*, int, const cx<double>*,
                                         hipStream_t, int, const cx<double>*, double*, int);
template int col_pass_lines<double>(int, int, int);
}  // namespace lp
