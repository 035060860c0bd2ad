// Host enumeration of the transform engine's index rules, compiled from the
// library's own headers (hipcc, host pass only) by tests/test_engine_bounds.py.
// For every supported length and element type (and every alternative FP32
// schedule of the autotuner) it checks, using the same
// constexpr schedules, helpers and launch configurations the kernels use:
//  * half-input prefetch (persistent row and column passes) and half-output
//    early loads (phase-gradient epilogue): every index in [0, n/2), each
//    element exactly once, only by threads that exist;
//  * every stage's LDS reads and writes stay inside the padded line, and the
//    strided forms the engine uses (one padded base plus compile-time
//    strides) address exactly the padded element;
//  * each launch configuration fits the LDS and thread limits;
//  * the persistent work split and the XCD remap cover each workgroup and
//    work item exactly once.
#include <cstdio>
#include <vector>

#include "fft_kernels.hpp"

using namespace lp;

static int failures = 0;
static void fail(const char* what, int n, int esz, int a = 0, int b = 0) {
  if (failures < 40) std::fprintf(stderr, "n=%d esz=%d: %s (%d, %d)\n", n, esz, what, a, b);
  ++failures;
}

template <class S, int s>
static void stage_lds(int esz) {
  constexpr int R = S::rad[s];
  constexpr int nr = S::n / R;
  constexpr int Ns = S::ns(s);
  constexpr int threads = S::threads;
  if (nr > threads) fail("stage has more butterflies than threads", S::n, esz, s, nr);
  for (int j = 0; j < nr; ++j) {
    for (int r = 0; r < R; ++r) {
      const int rd = j + r * nr;
      if (rd < 0 || rd >= S::n || S::pad(rd) >= S::line_elems) fail("stage read out of line", S::n, esz, s, rd);
      if (S::stride_pad(nr) && S::pad(j) + r * S::pstride(nr) != S::pad(rd))
        fail("strided read address", S::n, esz, s, rd);
      const int k = j % Ns, q = j / Ns;
      const int wr = q * Ns * R + k + r * Ns;
      if (wr < 0 || wr >= S::n || S::pad(wr) >= S::line_elems) fail("stage write out of line", S::n, esz, s, wr);
      if (Ns > 1 && S::stride_pad(Ns) && S::pad(q * Ns * R + k) + r * S::pstride(Ns) != S::pad(wr))
        fail("strided write address", S::n, esz, s, wr);
      if (Ns == 1 && S::contiguous_pad(R) && S::pad(q * R) + r != S::pad(wr))
        fail("contiguous write address", S::n, esz, s, wr);
    }
  }
}

template <class S, int... I>
static void all_stages(int esz, std::integer_sequence<int, I...>) {
  (stage_lds<S, I>(esz), ...);
}

template <class H>
static void half_cover(const char* what, int n, int esz, int threads, bool (*active)(int)) {
  std::vector<int> hits(n / 2, 0);
  for (int j = 0; j < threads; ++j) {
    if (!active(j)) continue;
    for (int r = 0; r < H::R; ++r) {
      const int i = H::index(j, r);
      if (i < 0 || i >= n / 2) {
        fail(what, n, esz, j, i);
        continue;
      }
      ++hits[i];
    }
  }
  for (int i = 0; i < n / 2; ++i)
    if (hits[i] != 1) fail(what, n, esz, i, hits[i]);
}

template <class S>
static bool hi_loads(int j) { return HalfIn<S>::loads(j); }
template <class S>
static bool ho_stores(int j) { return HalfOut<S>::stores(j); }

template <typename T, class S, int C, bool COL>
static void launch_fits(const char* what) {
  constexpr int LS = line_stride<S, C, COL>();
  if (LS < S::line_elems) fail("line stride below the padded line", S::n, (int)sizeof(T), C, LS);
  if ((long)C * LS * (long)sizeof(cx<T>) > kLdsBytes) fail(what, S::n, (int)sizeof(T), C, LS);
  if (C * S::threads > 1024) fail("workgroup above 1024 threads", S::n, (int)sizeof(T), C, S::threads);
}

template <typename T, class S>
static void check_len() {
  const int esz = (int)sizeof(T);
  all_stages<S>(esz, std::make_integer_sequence<int, S::nst>{});
  if (S::rad[0] % 2 == 0) half_cover<HalfIn<S>>("half-input prefetch", S::n, esz, S::threads, hi_loads<S>);
  if (S::rad[S::nst - 1] % 2 == 0)
    half_cover<HalfOut<S>>("half-output early load", S::n, esz, S::threads, ho_stores<S>);
  using CF = Cfg<T, S, true>;
  if constexpr (CF::fits) {
    launch_fits<T, S, CF::C, true>("column pass LDS");
    launch_fits<T, S, variant_lines<S, CF::C>(1), true>("column variant 1 LDS");
    launch_fits<T, S, variant_lines<S, CF::C>(2), true>("column variant 2 LDS");
    using RC = RowCfg<T, S>;
    launch_fits<T, S, RC::C, true>("row pass LDS");
    launch_fits<T, S, row_lines_two_per_cu<T, S, RC::C>(), true>("two-per-CU row pass LDS");
    using BC = Cfg<T, S, true, 1, 1024>;
    launch_fits<T, S, BC::C, true>("Bluestein column LDS");
    launch_fits<T, S, row_lines_two_per_cu<T, S, BC::C>(), true>("Bluestein row LDS");
  }
}

static void check_split() {
  for (int cus : {1, 7, 8, 64, 255, 256}) {
    for (int items = 1; items <= 3000; items += (items < 300 ? 1 : 37)) {
      const PersistSplit sp = persist_split(items, cus);
      if (sp.groups > cus || sp.groups < 1) fail("persistent groups", items, cus, sp.groups, sp.per);
      // every workgroup's run [g per, min(g per + per, items)) is non-empty
      if ((long)(sp.groups - 1) * sp.per >= items || (long)sp.groups * sp.per < items)
        fail("persistent runs", items, cus, sp.groups, sp.per);
    }
  }
  for (int nb = 1; nb <= 4100; ++nb) {
    std::vector<char> seen(nb, 0);
    for (int i = 0; i < nb; ++i) {
      const int t = xcd_remap(i, nb);
      if (t < 0 || t >= nb || seen[t]) {
        fail("xcd remap is not a permutation", nb, 0, i, t);
        break;
      }
      seen[t] = 1;
    }
  }
}

int main() {
#define LP_CHECK(N, ...)                                  \
  check_len<float, SchedOf<float, Sched<__VA_ARGS__>>>(); \
  check_len<double, SchedOf<double, Sched<__VA_ARGS__>>>();
  LP_LENGTHS(LP_CHECK)
#undef LP_CHECK
  // the alternative schedules the autotuner may choose (FP32)
#define LP_CHECK_ALT(N, ...) check_len<float, Sched<__VA_ARGS__>>();
  LP_ALT_LENGTHS(LP_CHECK_ALT)
#undef LP_CHECK_ALT
  check_split();
  if (failures) {
    std::fprintf(stderr, "%d index check(s) failed\n", failures);
    return 1;
  }
  std::printf("engine index rules hold for every supported length\n");
  return 0;
}
