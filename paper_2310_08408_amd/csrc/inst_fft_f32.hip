// Plain transform kernels for element type float, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_fft_lines<float, -1>(int, bool, const cx<float>*, cx<float>*, Lines, Lines, int, int, int, float,
                                             int, const cx<float>*, hipStream_t);
template hipError_t launch_fft_lines<float, 1>(int, bool, const cx<float>*, cx<float>*, Lines, Lines, int, int, int, float,
                                            int, const cx<float>*, hipStream_t);
template hipError_t launch_rs_rows<float, -1>(int, const cx<float>*, cx<float>*, int64_t, int, int, float, int,
                                            const cx<float>*, hipStream_t, const cx<float>*, float*, int,
                                            const Slm<float>*);
template hipError_t launch_rs_rows<float, 1>(int, const cx<float>*, cx<float>*, int64_t, int, int, float, int,
                                           const cx<float>*, hipStream_t, const cx<float>*, float*, int,
                                            const Slm<float>*);
}  // namespace lp
