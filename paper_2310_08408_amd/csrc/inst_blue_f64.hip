// Bluestein zoom-transform kernels (rows and columns, with and without the
// fused SLM stage) for element type double, all supported lengths.
#include "fft_kernels.hpp"

namespace lp {
template hipError_t launch_bluestein<double>(int, bool, const cx<double>*, cx<double>*, Lines, Lines, int, int, int,
                                         const cx<double>*, const cx<double>*, const cx<double>*, int, const cx<double>*,
                                         hipStream_t, int, const cx<double>*, double*, int, const Slm<double>*);
}  // namespace lp
