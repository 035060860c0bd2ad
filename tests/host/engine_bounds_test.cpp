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
//    work item exactly once;
//  * the LDS twiddle tables of the FP32 row passes (TwLds) give every
//    twiddled stage's W^{k r}: the global table entries they copy have the
//    right exponents (one entry for the first twiddled stage, two whose
//    exponents add up for the second), and every entry is in range;
//  * the buffer resources of the persistent RS column pass (the same
//    arithmetic as k_rs_cols_persist): for every lines-per-workgroup
//    variant, column count and work item, each lane's prefetch loads, stores
//    and spectrum gathers (vector offset plus scalar offset) fall inside the
//    item's resource, whose first 4-column tile and extent lie inside the
//    workspace and the spectrum table.
#include <algorithm>
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

// Buffer regions of k_rs_cols_persist<T, S, C> over ncols columns (n_valid =
// n/2 rows kept, spectrum table of q = n/2 + 1 rows in 4-column tiles).
template <typename T, class S, int C>
static void col_buffers(int ncols) {
  using HI = HalfIn<S>;
  using HO = HalfOut<S>;
  const long es = (long)sizeof(cx<T>);
  const int n = S::n, n_valid = n / 2, q = n / 2 + 1;
  const long tiles_w = (ncols + kTile - 1) / kTile;  // workspace 4-column tiles
  for (int tile = 0; tile < ncols / C; ++tile) {
    const int k0 = tile * C;
    const int ntiles = ((k0 & 3) + C + 3) / 4;
    if ((k0 >> 2) + ntiles > tiles_w) fail("column resource past the last tile", n, (int)es, C, tile);
    const long rw = (long)ntiles * n_valid * kTile * es, rq = (long)ntiles * q * 4 * es;
    if (rw >= (1L << 31) || rq >= (1L << 31)) fail("column resource above 2 GiB", n, (int)es, C, tile);
    for (int c = 0; c < C; ++c) {
      const int ka = (k0 & 3) + c;
      const long lane = (long)(ka >> 2) * n_valid * kTile + (ka & 3);
      const long lane_q = (long)(ka >> 2) * q * 4 + (ka & 3);
      // the lane's column must be the one the flat layout gives
      const int kx = k0 + c;
      if (lane + (long)(k0 >> 2) * n_valid * kTile != (long)(kx >> kTileShift) * n_valid * kTile + (kx & (kTile - 1)))
        fail("column lane offset", n, (int)es, C, kx);
      for (int j = 0; j < S::threads; ++j) {
        const long vo = (lane + (long)j * kTile) * es;
        if (HI::loads(j))
          for (int r = 0; r < HI::R; ++r) {
            const long so = (long)(HI::index(j, r) - j) * kTile * es;
            if (vo > rw || vo + so + es > rw) fail("column prefetch outside its resource", n, (int)es, C, j);
          }
        if (HO::stores(j))
          for (int r = 0; r < HO::R; ++r) {
            const long so = (long)(HO::index(j, r) - j) * kTile * es;
            if (vo > rw || vo + so + es > rw) fail("column store outside its resource", n, (int)es, C, j);
          }
      }
      for (int i = 0; i < n; ++i) {
        const long o = (lane_q + (long)std::min(i, n - i) * 4) * es;
        if (o + es > rq) fail("spectrum gather outside its resource", n, (int)es, C, i);
      }
    }
  }
}

template <typename T, class S>
static void check_col_buffers() {
  if constexpr (cols_persistent<T, S>() && S::rad[0] % 2 == 0 && S::rad[S::nst - 1] % 2 == 0) {
    using CF = Cfg<T, S, true>;
    if constexpr (CF::fits) {
      constexpr int C0 = CF::C, C1 = variant_lines<S, C0>(1), C2 = variant_lines<S, C0>(2);
      for (int ncols : {16, 48, S::n, 2 * S::n}) {
        if (ncols % C0 == 0) col_buffers<T, S, C0>(ncols);
        if (ncols % C1 == 0) col_buffers<T, S, C1>(ncols);
        if (ncols % C2 == 0) col_buffers<T, S, C2>(ncols);
      }
    }
  }
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

// Exponent e (W_n^e) of entry x of the global per-thread FP32 table of S:
// stage 1 (Ns = R0) holds W_{R0 R1}^{k r} = W_n^{k r n / (R0 R1)} at k R1 + r,
// stage 2 (Ns = R0 R1) W_n^{k r} at R0 R1 + k R2 + r.
template <class S>
static long tw_exponent(int x) {
  constexpr int R0 = S::rad[0], R1 = S::rad[1], R2 = S::nst == 3 ? S::rad[2] : 1;
  if (x < R0 * R1) return (long)(x / R1) * (x % R1) * (S::n / (R0 * R1));
  const int y = x - R0 * R1;
  return (long)(y / R2) * (y % R2);
}

template <class S>
static void check_twlds() {
  using L = TwLds<S>;
  if constexpr (L::ok) {
    const int n = S::n, R0 = S::rad[0], R1 = S::rad[1];
    const int size = S::twsize(true);
    for (int e = 0; e < L::elems; ++e)
      if (L::src(e) < 0 || L::src(e) >= size) fail("LDS twiddle source out of table", n, 4, e, L::src(e));
    for (int k = 0; k < R0; ++k)
      for (int r = 0; r < R1; ++r) {
        const int a = L::at1(k, r);
        if (a < 0 || a >= L::elems) fail("LDS twiddle entry out of range", n, 4, k, r);
        else if (tw_exponent<S>(L::src(a)) % n != (long)k * r * (n / (R0 * R1)) % n)
          fail("first-stage LDS twiddle exponent", n, 4, k, r);
      }
    if constexpr (S::nst == 3) {
      for (int k = 0; k < R0 * R1; ++k)
        for (int r = 0; r < S::rad[2]; ++r) {
          const int h = L::at2_hi(k, r), l = L::at2_lo(k, r);
          if (h < 0 || h >= L::elems || l < 0 || l >= L::elems) {
            fail("LDS twiddle entry out of range", n, 4, k, r);
            continue;
          }
          if ((tw_exponent<S>(L::src(h)) + tw_exponent<S>(L::src(l))) % n != (long)k * r % n)
            fail("second-stage LDS twiddle exponent", n, 4, k, r);
        }
    }
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
#define LP_CHECK(N, ...)                                    \
  check_len<float, SchedOf<float, Sched<__VA_ARGS__>>>();   \
  check_len<double, SchedOf<double, Sched<__VA_ARGS__>>>(); \
  check_col_buffers<float, SchedOf<float, Sched<__VA_ARGS__>>>(); \
  check_twlds<SchedOf<float, Sched<__VA_ARGS__>>>();
  LP_LENGTHS(LP_CHECK)
#undef LP_CHECK
  // the alternative schedules the autotuner may choose (FP32)
#define LP_CHECK_ALT(N, ...) \
  check_len<float, Sched<__VA_ARGS__>>(); \
  check_col_buffers<float, Sched<__VA_ARGS__>>(); \
  check_twlds<Sched<__VA_ARGS__>>();
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
