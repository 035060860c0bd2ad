// Plain transform kernels for element type double, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_fft_lines<double, -1>(int, bool, const cx<double>*, cx<double>*, Lines, Lines, int, int, int, double,
                                             int, const cx<double>*, hipStream_t);
template hipError_t launch_fft_lines<double, 1>(int, bool, const cx<double>*, cx<double>*, Lines, Lines, int, int, int, double,
                                            int, const cx<double>*, hipStream_t);
template hipError_t launch_rs_rows<double, -1>(int, const cx<double>*, cx<double>*, int64_t, int, int, double, int,
                                            const cx<double>*, hipStream_t, const cx<double>*, double*, int,
                                            const Slm<double>*);
template hipError_t launch_rs_rows<double, 1>(int, const cx<double>*, cx<double>*, int64_t, int, int, double, int,
                                           const cx<double>*, hipStream_t, const cx<double>*, double*, int,
                                            const Slm<double>*);
}  // namespace lp
