// Host-side argument validation of the libprop C ABI: grid and parameter
// checks, transform-length planning, aliasing of device ranges and the
// sampling warning of the RS kernel.  Plain C++ (no HIP), so the checks can
// be built and exercised on the host alone, also under sanitizers.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <initializer_list>
#include <utility>
#include <vector>

#include "lengths.hpp"
#include "libprop.h"

namespace lp {

static const int kLengths[] = {
#define LP_LEN(N, ...) N,
    LP_LENGTHS(LP_LEN)
#undef LP_LEN
};

// Smallest supported transform length >= n, or -1.
inline int fft_len(int n) {
  if (n < 1) return -1;
  int best = -1;
  for (int v : kLengths)
    if (v >= n && (best < 0 || v < best)) best = v;
  return best;
}

inline bool is_finite(double v) { return std::isfinite(v); }

inline int check_grid(const prop_grid* g) {
  if (!g) return PROP_ENULL;
  if (g->nx < 1 || g->ny < 1) return PROP_ESHAPE;
  if (!(g->dx > 0) || !(g->dy > 0) || !is_finite(g->dx) || !is_finite(g->dy) || !is_finite(g->cx) || !is_finite(g->cy))
    return PROP_EPARAM;
  return PROP_OK;
}

inline int check_common(prop_dtype t, int32_t batch, double wl) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (batch < 0) return PROP_ESHAPE;
  if (!(wl > 0) || !is_finite(wl)) return PROP_EPARAM;
  return PROP_OK;
}

inline int check_lens(const prop_lens* lens) {
  if (!lens) return PROP_OK;
  if (!(lens->na > 0) || !(lens->na < 1) || !(lens->f > 0) || !is_finite(lens->f)) return PROP_EPARAM;
  return PROP_OK;
}

// RS and VRS transform lengths (2n - 1 per axis, padded) must be supported.
inline int check_rs_shape(const prop_grid* g) {
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  return PROP_OK;
}

// CZT Bluestein lengths (n_in + n_out - 1 per axis) must be supported.
inline int check_czt_shapes(const prop_grid* gi, const prop_grid* go) {
  if (fft_len(gi->nx + go->nx - 1) < 0 || fft_len(gi->ny + go->ny - 1) < 0) return PROP_ESHAPE;
  return PROP_OK;
}

inline size_t esize(prop_dtype t) { return t == PROP_C64 ? 8 : 16; }

// Byte ranges [a, a + na) and [b, b + nb) overlap.
inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// every output must be disjoint from every input and from each other
using Span = std::pair<const void*, size_t>;

inline int check_alias(const std::vector<Span>& ins, const std::vector<Span>& o) {
  for (size_t i = 0; i < o.size(); ++i) {
    for (auto& in : ins)
      if (overlap(o[i].first, o[i].second, in.first, in.second)) return PROP_EALIAS;
    for (size_t j = i + 1; j < o.size(); ++j)
      if (overlap(o[i].first, o[i].second, o[j].first, o[j].second)) return PROP_EALIAS;
  }
  return PROP_OK;
}

inline int check_alias(std::initializer_list<Span> ins, std::initializer_list<Span> outs) {
  return check_alias(std::vector<Span>(ins), std::vector<Span>(outs));
}

// Sampling reading of the RS kernel: exp(ikr) must be Nyquist-sampled at
// the largest lateral offset L = n d, i.e. a warning when 2 d > lambda and
// z < sqrt((2 L d / lambda)^2 - L^2) along some axis.
inline int sampling(const prop_grid* g, double wl, double z) {
  const int n[2] = {g->nx, g->ny};
  const double d[2] = {g->dx, g->dy};
  for (int a = 0; a < 2; ++a) {
    if (2.0 * d[a] <= wl) continue;
    const double L = n[a] * d[a];
    const double zmin = std::sqrt((2.0 * L * d[a] / wl) * (2.0 * L * d[a] / wl) - L * L);
    if (z < zmin) return PROP_WUNDERSAMPLED;
  }
  return PROP_OK;
}

}  // namespace lp
