// Bluestein zoom-transform kernels (rows and columns, with and without the
// fused SLM stage) for element type float, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_bluestein<float>(int, bool, const cx<float>*, cx<float>*, Lines, Lines, int, int, int,
                                         const cx<float>*, const cx<float>*, const cx<float>*, int, const cx<float>*,
                                         hipStream_t, int, const cx<float>*, float*, int, const Slm<float>*);
}  // namespace lp
