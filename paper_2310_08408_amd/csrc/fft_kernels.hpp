// Transform kernels (templated on element type, radix schedule and lines per
// workgroup) and their host launchers, which switch over the supported
// lengths.  Included by the per-type instantiation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.hpp"

namespace lp {

constexpr int kLdsBytes = 160 * 1024;  // LDS per CU (and per workgroup) on gfx950
constexpr int kColThreads = 1024;      // thread cap of column-pass workgroups

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Element stride between the LDS lines of one workgroup.  Lanes of a
// half-wave that belong to different lines must hit different banks:
// column mode interleaves C lines lane by lane, so lines are offset by
// 32/C elements modulo 32; row mode with T < 32 threads per line packs
// 32/T lines per half-wave, so lines are offset by T.
template <class S, int C, bool COL>
constexpr int line_stride() {
  constexpr int base = (S::line_elems + 31) / 32 * 32;
  constexpr int off = C <= 1 ? 1 : (COL ? (32 / (C < 32 ? C : 32)) % 32 : (S::threads < 32 ? S::threads : 1));
  return base + off;
}

// Waves per SIMD that the LDS footprint of a workgroup allows (at most 8):
// asking the compiler for this occupancy caps its register budget so that
// registers do not become the tighter limit.
template <typename T, class S, int C, bool COL, int LPI = 1, int CAP = 4>
constexpr int waves_per_eu() {
  constexpr int threads = C * S::threads * LPI;
  constexpr int wg_waves = (threads + 63) / 64;
  constexpr int lds = C * LPI * line_stride<S, C, COL>() * (int)sizeof(cx<T>);
  constexpr int wgs = kLdsBytes / (lds > 0 ? lds : 1);
  constexpr int w = (wgs * wg_waves) / 4;
  constexpr int cap = sizeof(T) == 4 ? CAP : 1;  // FP64 kernels: no occupancy request
  return w < 1 ? 1 : (w > cap ? cap : w);
}

// Lines per workgroup of a row pass that interleaves C0 lines lane by lane.
// Rows are contiguous, so fewer lines per workgroup still move whole row
// segments; halving (down to 2) until two workgroups fit in a CU's LDS
// lets one workgroup's barrier waits overlap the other's arithmetic.  At
// 4096 points this turns one 4-line workgroup per CU into two 2-line ones
// (Bluestein rows 15% faster, RS inverse rows 6%); a single line per
// workgroup loses again (each lane then needs its own twiddle run).
template <typename T, class S, int C0>
constexpr int row_lines_two_per_cu() {
  constexpr int line = ((S::line_elems + 31) / 32 * 32 + 32) * (int)sizeof(cx<T>);  // bound on one LDS line
  int c = C0;
  while (c > 2 && c % 2 == 0 && 2 * c * line > kLdsBytes) c /= 2;  // stays a divisor of C0
  return c;
}

// Lines per workgroup.  Column passes pack adjacent columns (wide coalesced
// segments) up to the LDS and thread limits; row passes aim at >= 256
// threads with at most half the LDS (two workgroups per CU).
template <typename T, class S, bool COL, int LINES_PER_ITEM = 1, int COL_THREADS = kColThreads>
struct Cfg {
  static constexpr int line_bytes = (S::line_elems + 64) * (int)sizeof(cx<T>) * LINES_PER_ITEM;
  static constexpr int max_threads = COL ? COL_THREADS : 1024;
  static constexpr int c_col = cmax(1, cmin(cmin(16, max_threads / (S::threads * LINES_PER_ITEM)), kLdsBytes / line_bytes));
  static constexpr int c_row =
      cmax(1, cmin(cmin(cmax(1, 256 / (S::threads * LINES_PER_ITEM)), (kLdsBytes / 2) / line_bytes),
                   max_threads / (S::threads * LINES_PER_ITEM)));
  static constexpr int C = COL ? c_col : c_row;
  static constexpr int threads = C * S::threads * LINES_PER_ITEM;
  static constexpr bool fits = line_bytes <= kLdsBytes && S::threads * LINES_PER_ITEM <= 1024;
};

// Tunable launch variants of the column passes: variant v runs C >> v lines
// per workgroup (at least 1) instead of the built-in C, for lengths >= 512.
// Every variant computes bit-identical results (only the assignment of
// lines to workgroups changes); the library's autotuner picks among them.
constexpr int kTuneMinLength = 512;
template <class S, int C0>
constexpr int variant_lines(int v) {
  return S::n >= kTuneMinLength ? cmax(1, C0 >> v) : C0;
}

// Workgroup i is dispatched to XCD i % 8; give each XCD a contiguous range
// of tiles so that neighbouring lines (adjacent columns) share one L2.
__host__ __device__ __forceinline__ int xcd_remap(int i, int nb) {
  const int q = nb >> 3, r = nb & 7, x = i & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

// Work split of a persistent pass over `items` work items: `per` items per
// workgroup, `groups` workgroups, at most one per compute unit; every
// workgroup gets a non-empty contiguous run.
struct PersistSplit {
  int per, groups;
};
__host__ __device__ constexpr PersistSplit persist_split(int items, int cus) {
  const int per = (items + cus - 1) / cus;
  return PersistSplit{per, (items + per - 1) / per};
}

// Compute units of the current device (cached per device).
inline int cu_count() {
  static int counts[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!counts[dev]) {
    int v = 0;
    counts[dev] = (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                      ? v
                      : 256;
  }
  return counts[dev];
}

// FP32 row passes (RS rows, Bluestein rows) of two- and three-stage
// schedules take their twiddles from LDS tables (TwLds) instead of the
// per-thread global runs, whose L2 round trip every wave of a workgroup
// waits for at once -- where the tables keep the workgroups per CU that the
// line buffers allow.  At 2048^2, batch 8 (4096 points): Bluestein rows 285
// -> 228 us, RS inverse rows 226 -> 213, persistent forward rows 164 -> 155.
// The column passes keep the global table: there the LDS form measured
// slower (RS columns 422 -> 435 us; Bluestein columns 319 -> 349, where it
// also spills).
template <typename T, class S, int C, bool ILV>
constexpr bool tw_lds() {
  if constexpr (!std::is_same<T, float>::value || !TwLds<S>::ok) {
    return false;
  } else {
    constexpr int base = C * line_stride<S, C, ILV>() * (int)sizeof(cx<T>);
    constexpr int with = base + TwLds<S>::elems * (int)sizeof(cx<T>);
    return with <= kLdsBytes && kLdsBytes / with == kLdsBytes / base;
  }
}

// The twiddles a pass reads: with TL the LDS table pair after the line
// buffers (filled here; the caller's next barrier publishes it), else the
// global table.
template <bool TL, class S, typename T>
__device__ __forceinline__ const cx<T>* tw_source(cx<T>* tl, const cx<T>* tw, int nthreads) {
  if constexpr (TL) {
    TwLds<S>::fill(tl, tw, threadIdx.x, nthreads);
    return tl;
  } else {
    return tw;
  }
}

// Streaming accesses without cache retention (non-temporal): for passes in
// which each element is touched once and one workgroup consumes whole
// lines, so that the transform's twiddle tables stay cached instead.  Not
// for passes whose lines are shared by neighbouring workgroups.
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  using V2 = T __attribute__((ext_vector_type(2)));
  const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
  return mk<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> a) {
  using V2 = T __attribute__((ext_vector_type(2)));
  V2 v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<V2*>(p));
}

// Optional fused SLM phase gradient on a pass's store: grad = Im(g conj u)
// for the stored value g (added to grad when acc), at the output element.
template <typename T>
struct PhaseGrad {
  const cx<T>* u = nullptr;
  T* grad = nullptr;
  int acc = 0;
  __device__ __forceinline__ void put(int64_t o, cx<T> g) const {
    const cx<T> v = u[o];
    const T d = g.y * v.x - g.x * v.y;
    grad[o] = acc ? grad[o] + d : d;
  }
};

// The phase-gradient epilogue of an exact-half line pass whose last stage
// (radix RL) stores outputs j + r n/RL, r < RL/2: the field values it needs
// and the gradient it accumulates into are loaded when the kernel starts, so
// their HBM latency overlaps the transform instead of stalling every store
// at the end.  FP32 with a first radix of at most 16 only: there the
// registers fit beside the transform.
template <typename T, class S, bool EXACT_HALF>
constexpr bool pg_preload() {
  return EXACT_HALF && sizeof(T) == 4 && S::rad[0] <= 16;
}
template <typename T, class S, bool ON>
struct PhaseGradPre {
  using HO = HalfOut<S>;
  static constexpr int nr = HO::nr, P = ON ? HO::R : 1;
  cx<T> u[P];
  T g[P];
  template <class Off>
  __device__ __forceinline__ void load(const PhaseGrad<T>& pg, int j, Off off) {
    if constexpr (ON) {
      if (pg.grad && HO::stores(j)) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
          const int64_t o = off(HO::index(j, r));
          u[r] = pg.u[o];
          g[r] = pg.acc ? pg.grad[o] : T(0);
        }
      }
    }
  }
  // store of output i (= j + r n/RL) at offset o
  __device__ __forceinline__ void put(const PhaseGrad<T>& pg, int i, int j, int64_t o, cx<T> v) const {
    if constexpr (ON) {
      const int r = (i - j) / nr;
      const T d = v.y * u[r].x - v.x * u[r].y;
      pg.grad[o] = pg.acc ? g[r] + d : d;
    } else {
      pg.put(o, v);
    }
  }
};

// Factor of the fused SLM stage (Slm) at field element (row, col) of batch
// item b, and the adjoint store of a pass that ends in it: g_V = g_U
// conj(factor), with the phase gradient Im(g_V conj V) when requested.
template <typename T> __device__ __forceinline__ void slm_sincos(T x, T* s, T* c);
template <> __device__ __forceinline__ void slm_sincos<float>(float x, float* s, float* c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void slm_sincos<double>(double x, double* s, double* c) { sincos(x, s, c); }

template <typename T>
__device__ __forceinline__ cx<T> slm_factor(const Slm<T>& st, int b, int row, int col) {
  cx<T> f = mk<T>(T(1), T(0));
  if (st.phase) {
    T sn, cs;
    slm_sincos<T>(st.phase[b * st.pbs + (int64_t)row * st.nx + col], &sn, &cs);
    f = mk<T>(cs, sn);
  }
  if (st.lx) f = cmul(f, cmul(st.lx[col], st.ly[row]));
  return f;
}

template <typename T>
__device__ __forceinline__ cx<T> slm_adjoint_store(const Slm<T>& st, const PhaseGrad<T>& pg, cx<T>* out, int b,
                                                   int row, int col, int64_t o, cx<T> g) {
  const cx<T> gv = cmulc(g, slm_factor(st, b, row, col));
  if (out) out[o] = gv;
  if (pg.grad) pg.put(o, gv);
  return gv;
}

template <typename T> __device__ __forceinline__ cx<T> czero() { return mk<T>(T(0), T(0)); }

// The fused SLM stage on the stores of an exact-half inverse row pass,
// with its phase loaded when the kernel starts (as PhaseGradPre does for the
// phase-gradient epilogue) at the indices the last stage stores (j + r n/RL,
// r < RL/2), so that the load's HBM latency overlaps the transform.  The
// store then forms the same products as slm_adjoint_store.  ON = false:
// slm_adjoint_store at the store.
template <typename T, class S, bool ON>
struct SlmPre {
  using HO = HalfOut<S>;
  static constexpr int nr = HO::nr, P = ON ? HO::R : 1;
  T ph[P];
  __device__ __forceinline__ void load(const Slm<T>& st, const PhaseGrad<T>& pg, int b, int row, int j,
                                       int64_t frow) {
    if constexpr (ON) {
      if (HO::stores(j)) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
          const int i = HO::index(j, r);
          ph[r] = st.phase ? st.phase[b * st.pbs + (int64_t)row * st.nx + i] : T(0);
        }
      }
    }
  }
  __device__ __forceinline__ void store(const Slm<T>& st, const PhaseGrad<T>& pg, cx<T>* out, int b, int row,
                                        int i, int j, int64_t o, cx<T> g) const {
    if constexpr (ON) {
      const int r = (i - j) / nr;
      cx<T> f = mk<T>(T(1), T(0));
      if (st.phase) {
        T sn, cs;
        slm_sincos<T>(ph[r], &sn, &cs);
        f = mk<T>(cs, sn);
      }
      if (st.lx) f = cmul(f, cmul(st.lx[i], st.ly[row]));
      const cx<T> gv = cmulc(g, f);
      if (out) out[o] = gv;
      if (pg.grad) pg.put(o, gv);
    } else {
      slm_adjoint_store(st, pg, out, b, row, i, o, g);
    }
  }
};

// address of element i of line l of batch item b
template <bool COL>
__device__ __forceinline__ int64_t line_off(const Lines& L, int b, int l, int i) {
  return COL ? (int64_t)b * L.bstride + (int64_t)i * L.pitch + l : (int64_t)b * L.bstride + (int64_t)l * L.pitch + i;
}

// ------------------------------------------------------------ FFT lines --
template <typename T, int DIR, bool COL, class S, int C>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, COL>())) void k_fft_lines(const cx<T>* in, cx<T>* out, Lines li, Lines lo,
                                                              int nlines, int n_in, int n_out, T scale, int tiles,
                                                              const cx<T>* __restrict__ tw) {
  constexpr int LS = line_stride<S, C, COL>();
  __shared__ cx<T> smem[C * LS];
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int b = id / tiles, tile = id - b * tiles;
  const int c = COL ? (int)(threadIdx.x % C) : (int)(threadIdx.x / S::threads);
  const int j = COL ? (int)(threadIdx.x / C) : (int)(threadIdx.x % S::threads);
  const int l = tile * C + c;
  const bool valid = l < nlines;
  cx<T>* lds = smem + c * LS;
  auto load = [&](int i) -> cx<T> {
    cx<T> v = czero<T>();
    if (valid && i < n_in) v = in[line_off<COL>(li, b, l, i)];
    return v;
  };
  auto store = [&](int i, cx<T> v) {
    if (valid && i < n_out) out[line_off<COL>(lo, b, l, i)] = cscale(v, scale);
  };
  fft_line<T, DIR, S>(lds, tw, j, load, store);
}

template <typename T, int DIR, bool COL, class S>
hipError_t launch_fft_lines_s(const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in, int n_out,
                              T scale, int batch, const cx<T>* tw, hipStream_t s) {
  using CF = Cfg<T, S, COL>;
  if constexpr (!CF::fits) {
    return hipErrorInvalidValue;
  } else {
    const int tiles = (nlines + CF::C - 1) / CF::C;
    hipLaunchKernelGGL((k_fft_lines<T, DIR, COL, S, CF::C>), dim3(tiles * batch), dim3(CF::threads), 0, s, in, out,
                       li, lo, nlines, n_in, n_out, scale, tiles, tw);
    return hipGetLastError();
  }
}

template <typename T, int DIR>
hipError_t launch_fft_lines(int n, bool col, const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in,
                            int n_out, T scale, int batch, const cx<T>* tw, hipStream_t s) {
  if (nlines <= 0 || batch <= 0) return hipSuccess;
  switch (n) {
#define LP_CASE(N, ...)                                                                                          \
  case N:                                                                                                        \
    return col ? launch_fft_lines_s<T, DIR, true, SchedOf<T, Sched<__VA_ARGS__>>>(in, out, li, lo, nlines, n_in, n_out, scale, \
                                                                     batch, tw, s)                               \
               : launch_fft_lines_s<T, DIR, false, SchedOf<T, Sched<__VA_ARGS__>>>(in, out, li, lo, nlines, n_in, n_out,     \
                                                                      scale, batch, tw, s);
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// A read-only table (kernel spectrum, twiddles) boxed in a struct.  Passed
// as a __restrict__ pointer instead, the compiler may treat its loads as
// invariant and lift them across barriers: that hides their latency while
// registers last, and spills where they do not.  Boxed, the loads stay where
// the code issues them.
template <typename T> struct TableBox { const cx<T>* p; };
template <typename T, bool BOX>
using TableArg = std::conditional_t<BOX, TableBox<T>, const cx<T>* __restrict__>;
template <typename T> __device__ __forceinline__ const cx<T>* table_ptr(TableBox<T> b) { return b.p; }
template <typename T> __device__ __forceinline__ const cx<T>* table_ptr(const cx<T>* p) { return p; }

// ------------------------------------------------------ RS row passes --
// Forward (DIR = -1): row y of a contiguous field, zero-padded from n_io to
// n, transformed into the tiled workspace.  Inverse (DIR = +1): workspace
// row y transformed back, the first n_io outputs scaled into the field.
// A workgroup holds C rows with lanes interleaved across them.  With
// C >= kTile one wave's store or load covers whole tiles (kTile rows x kTile
// columns, contiguous) on the workspace side and C row segments on the field
// side; the exact inverse pass may take fewer rows (row_lines_two_per_cu),
// neighbouring workgroups then sharing tiles through the L2.
// HALF prunes the zero half of the forward input / the unused half of the
// inverse output at compile time.
template <typename T, class S>
struct RowCfg {
  using CF = Cfg<T, S, false>;
  static constexpr int line_bytes = (S::line_elems + 64) * (int)sizeof(cx<T>);
  static constexpr int C = cmax(1, cmin(cmin(cmax(kTile, CF::c_row), kLdsBytes / line_bytes), 1024 / S::threads));
  static constexpr int threads = C * S::threads;
  static constexpr bool fits = CF::fits;
};

// EXACT (with HALF): the valid length is exactly n/2 and the line count a
// multiple of C, so no load or store needs a guard; the guards' branches
// otherwise split every access into its own exec-masked block.
// PG = false: an instance without the phase-gradient epilogue, for launches
// that have none (its early loads would hold 24 VGPRs for nothing).
// STAGE: the fused SLM stage of a plan setup (Slm) on the loads (forward)
// or the stores (inverse).
template <typename T, int DIR, class S, int C, bool HALF, bool EXACT = false, bool PG = true, bool STAGE = false>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, true>())) void k_rs_rows(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int64_t w_bstride, int nrows, int n_io, T scale, int tiles,
    const cx<T>* __restrict__ tw_g, PhaseGrad<T> pg, Slm<T> st) {
  constexpr int LS = line_stride<S, C, true>();
  constexpr bool TL = tw_lds<T, S, C, true>();
  __shared__ cx<T> smem[C * LS + (TL ? TwLds<S>::elems : 0)];
  // (the first stage's barrier publishes the LDS twiddles before their use)
  const cx<T>* tw = tw_source<TL, S>(smem + C * LS, tw_g, C * S::threads);
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int b = id / tiles, tile = id - b * tiles;
  const int c = (int)(threadIdx.x % C), j = (int)(threadIdx.x / C);
  const int y = tile * C + c;
  const bool valid = EXACT || y < nrows;
  cx<T>* lds = smem + c * LS;
  const int64_t tst = (int64_t)nrows * kTile;  // elements between tiles
  const int64_t frow = ((int64_t)b * nrows + y) * n_io;
  const int64_t wrow = b * w_bstride + (int64_t)y * kTile;
  auto widx = [&](int i) { return wrow + (int64_t)(i >> kTileShift) * tst + (i & (kTile - 1)); };
  if constexpr (DIR < 0) {
    auto load = [&](int i) -> cx<T> {
      cx<T> v = czero<T>();
      if (valid && (EXACT || i < n_io)) {
        v = in[frow + i];
        if constexpr (STAGE) v = cmul(v, slm_factor(st, b, y, i));
      }
      return v;
    };
    auto store = [&](int i, cx<T> v) {
      if (valid) out[widx(i)] = v;
    };
    fft_line<T, -1, S, HALF, false, TL>(lds, tw, j, load, store);
  } else {
    auto load = [&](int i) -> cx<T> {
      cx<T> v = czero<T>();
      if (valid) v = in[widx(i)];
      return v;
    };
    PhaseGradPre<T, S, PG && !STAGE && pg_preload<T, S, EXACT && HALF>()> pre_pg;
    pre_pg.load(pg, j, [&](int i) { return frow + i; });
    SlmPre<T, S, STAGE && pg_preload<T, S, EXACT && HALF>()> pre_st;
    if constexpr (STAGE) pre_st.load(st, pg, b, y, j, frow);
    auto store = [&](int i, cx<T> v) {
      if (valid && (EXACT || i < n_io)) {
        const cx<T> g = cscale(v, scale);
        if constexpr (STAGE) {
          pre_st.store(st, pg, out, b, y, i, j, frow + i, g);
        } else {
          if (out) out[frow + i] = g;
          if constexpr (PG) {
            if (pg.grad) pre_pg.put(pg, i, j, frow + i, g);
          }
        }
      }
    };
    fft_line<T, 1, S, false, HALF, TL>(lds, tw, j, load, store);
  }
}

// Forward exact-half row pass in persistent form (FP32 tables in per-thread
// runs, first radix <= 16): one workgroup per CU walks a contiguous run of
// (batch item, row tile) items and loads the next item's row segment into
// registers while it transforms the current one.  The engine reads the half
// input as elements j + r n/R0 (r < R0/2) of the threads j < n/R0 only, so
// those threads alone prefetch, each its own elements.
template <typename T, class S, int C, bool STAGE = false>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, true>())) void k_rs_rows_fwd_persist(
    const cx<T>* in, cx<T>* out, int64_t w_bstride, int nrows, int n_io, int tiles, int items, int per,
    TableBox<T> tw_, Slm<T> st) {
  constexpr int LS = line_stride<S, C, true>();
  constexpr bool TL = tw_lds<T, S, C, true>();
  __shared__ cx<T> smem[C * LS + (TL ? TwLds<S>::elems : 0)];
  // (the first stage's barrier publishes the LDS twiddles before their use)
  const cx<T>* tw = tw_source<TL, S>(smem + C * LS, tw_.p, C * S::threads);
  using HI = HalfIn<S>;
  constexpr int RIN = HI::R;
  const int chunk = xcd_remap(blockIdx.x, gridDim.x);
  const int first = chunk * per, last = min(first + per, items);
  const int c = (int)(threadIdx.x % C), j = (int)(threadIdx.x / C);
  cx<T>* lds = smem + c * LS;
  const int64_t tst = (int64_t)nrows * kTile;
  const bool loader = HI::loads(j);
  auto frow = [&](int id) -> int64_t {
    const int b = id / tiles, y = (id - b * tiles) * C + c;
    return ((int64_t)b * nrows + y) * n_io;
  };
  cx<T> nxt[RIN];
  if (loader && first < last) {
    const cx<T>* src = in + frow(first);
#pragma unroll
    for (int r = 0; r < RIN; ++r) nxt[r] = src[HI::index(j, r)];
  }
  for (int id = first; id < last; ++id) {
    cx<T> cur[RIN];
#pragma unroll
    for (int r = 0; r < RIN; ++r) cur[r] = nxt[r];
    if (loader && id + 1 < last) {
      const cx<T>* src = in + frow(id + 1);
#pragma unroll
      for (int r = 0; r < RIN; ++r) nxt[r] = src[HI::index(j, r)];
    }
    const int b = id / tiles, y = (id - b * tiles) * C + c;
    const int64_t wrow = b * w_bstride + (int64_t)y * kTile;
    // the first stage asks for i = HI::index(j, r): register r of cur
    auto load = [&](int i) -> cx<T> {
      if constexpr (STAGE) return cmul(cur[(i - j) / HI::nr], slm_factor(st, b, y, i));
      return cur[(i - j) / HI::nr];
    };
    auto store = [&](int i, cx<T> v) { out[wrow + (int64_t)(i >> kTileShift) * tst + (i & (kTile - 1))] = v; };
    fft_line<T, -1, S, true, false, TL>(lds, tw, j, load, store);
  }
}

template <typename T, int DIR, class S, bool STAGE>
hipError_t launch_rs_rows_st(const cx<T>* in, cx<T>* out, int64_t w_bstride, int nrows, int n_io, T scale, int batch,
                             const cx<T>* tw, hipStream_t s, PhaseGrad<T> pg, Slm<T> st) {
  using RC = RowCfg<T, S>;
  if constexpr (!RC::fits) {
    return hipErrorInvalidValue;
  } else {
    constexpr int C = RC::C;
    const int tiles = (nrows + C - 1) / C;
    constexpr bool can_half = S::rad[0] % 2 == 0 && S::rad[S::nst - 1] % 2 == 0;
    if constexpr (can_half) {
      if (2 * n_io == S::n && nrows % C == 0) {
        // (with the fused SLM stage the persistent form's prefetch registers
        // spill next to the stage's sincos: the plain instance runs instead)
        if constexpr (DIR < 0 && tw_per_thread<T>() && S::rad[0] <= 16 && !STAGE) {
          const int items = tiles * batch;
          const PersistSplit sp = persist_split(items, cu_count());
          hipLaunchKernelGGL((k_rs_rows_fwd_persist<T, S, C>), dim3(sp.groups), dim3(RC::threads), 0, s, in, out,
                             w_bstride, nrows, n_io, tiles, items, sp.per, TableBox<T>{tw}, st);
        } else {
          // rows need not fill whole workspace tiles: C2 may be below kTile.
          // With the phase-gradient epilogue fused, C lines measure faster
          // (4096: 248 against 257 us; plain: 218 against 212 us at C2).
          constexpr int C2 = row_lines_two_per_cu<T, S, C>();
          if (C2 != C && !pg.grad && !STAGE) {
            const int tiles2 = nrows / C2;
            hipLaunchKernelGGL((k_rs_rows<T, DIR, S, C2, true, true, false>), dim3(tiles2 * batch),
                               dim3(C2 * S::threads), 0, s, in, out, w_bstride, nrows, n_io, scale, tiles2, tw, pg,
                               st);
          } else {
            hipLaunchKernelGGL((k_rs_rows<T, DIR, S, C, true, true, true, STAGE>), dim3(tiles * batch),
                               dim3(RC::threads), 0, s, in, out, w_bstride, nrows, n_io, scale, tiles, tw, pg, st);
          }
        }
        return hipGetLastError();
      }
      if (2 * n_io <= S::n) {
        hipLaunchKernelGGL((k_rs_rows<T, DIR, S, C, true, false, true, STAGE>), dim3(tiles * batch),
                           dim3(RC::threads), 0, s, in, out, w_bstride, nrows, n_io, scale, tiles, tw, pg, st);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_rs_rows<T, DIR, S, C, false, false, true, STAGE>), dim3(tiles * batch), dim3(RC::threads),
                       0, s, in, out, w_bstride, nrows, n_io, scale, tiles, tw, pg, st);
    return hipGetLastError();
  }
}

template <typename T, int DIR, class S>
hipError_t launch_rs_rows_s(const cx<T>* in, cx<T>* out, int64_t w_bstride, int nrows, int n_io, T scale, int batch,
                            const cx<T>* tw, hipStream_t s, PhaseGrad<T> pg, const Slm<T>* slm) {
  if (slm && slm->active())
    return launch_rs_rows_st<T, DIR, S, true>(in, out, w_bstride, nrows, n_io, scale, batch, tw, s, pg, *slm);
  return launch_rs_rows_st<T, DIR, S, false>(in, out, w_bstride, nrows, n_io, scale, batch, tw, s, pg, Slm<T>{});
}

template <typename T, int DIR>
hipError_t launch_rs_rows(int n, const cx<T>* in, cx<T>* out, int64_t w_bstride, int nrows, int n_io, T scale,
                          int batch, const cx<T>* tw, hipStream_t s, const cx<T>* pg_u, T* pg_grad, int pg_acc,
                          const Slm<T>* slm) {
  if (nrows <= 0 || batch <= 0) return hipSuccess;
  PhaseGrad<T> pg;
  pg.u = pg_u;
  pg.grad = pg_grad;
  pg.acc = pg_acc;
  switch (n) {
#define LP_CASE(N, ...) \
  case N: return launch_rs_rows_s<T, DIR, SchedOf<T, Sched<__VA_ARGS__>>>(in, out, w_bstride, nrows, n_io, scale, batch, tw, s, pg, slm);
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// ------------------------------------------------- kernel-spectrum access --
// Half table (rows 0..My/2, 4-column tiles) of an RS-type kernel spectrum
// with parity in ky: kinds 0 (H) and 1 ((X/z) H) even, kind 2 ((Y/z) H) odd.
template <typename T>
__device__ __forceinline__ cx<T> spec_at(const cx<T>* __restrict__ Sq, int kind, int kx, int ky, int Mx, int My) {
  const int qy = min(ky, My - ky);
  cx<T> h = Sq[(int64_t)(kx >> 2) * (My / 2 + 1) * 4 + qy * 4 + (kx & 3)];
  if (kind == 2 && ky > My / 2) { h.x = -h.x; h.y = -h.y; }
  return h;
}

// ------------------------------------------------------ RS column pass --
// In place on columns kx of W: forward transform of the zero-padded column,
// multiply by the kernel spectrum (conjugated for the adjoint), inverse
// transform, keep the first n_valid rows.
// EXACT: as for the row pass.  Its unguarded loads are scheduled early by
// themselves, so the tables come boxed (lifting them as well would spill).
template <typename T, class S, int C, bool HALF, bool EXACT = false>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, true>())) void k_rs_cols(cx<T>* W, int64_t bstride, int ncols,
                                                            int n_valid, TableArg<T, EXACT> Sq_, int Mx,
                                                            int conj_spec, int tiles, TableArg<T, EXACT> tw_) {
  const cx<T>* Sq = table_ptr<T>(Sq_);
  const cx<T>* tw = table_ptr<T>(tw_);
  constexpr int LS = line_stride<S, C, true>();
  __shared__ cx<T> smem[C * LS];
  constexpr int My = S::n;
  // batch-minor order: the batch items of one column tile run side by side
  // on one XCD and share the kernel-spectrum lines in its L2
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int nb = gridDim.x / tiles;
  const int tile = id / nb, b = id - tile * nb;
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  const int kx = tile * C + c;
  const bool valid = EXACT || kx < ncols;
  cx<T>* lds = smem + c * LS;
  cx<T>* col = W + b * bstride + (int64_t)(kx >> kTileShift) * n_valid * kTile + (kx & (kTile - 1));
  const cx<T>* sq = Sq + (valid ? (int64_t)(kx >> 2) * (My / 2 + 1) * 4 + (kx & 3) : 0);
  auto load = [&](int i) -> cx<T> {
    cx<T> v = czero<T>();
    if (valid && (EXACT || i < n_valid)) v = load_stream(&col[i * kTile]);
    return v;
  };
  auto mult = [&](int i, cx<T> v) -> cx<T> {
    cx<T> h = czero<T>();
    if (valid) h = sq[min(i, My - i) * 4];
    if (conj_spec) h.y = -h.y;  // one product, not two and a select
    return cmul(v, h);
  };
  auto store = [&](int i, cx<T> v) {
    if (valid && (EXACT || i < n_valid)) store_stream(&col[i * kTile], v);
  };
  conv_line<T, S, HALF, HALF>(lds, tw, j, load, mult, store);
}

// Exact-half column pass (valid length n/2, column count a multiple of C)
// in persistent form, for FP32 schedules whose first and last radix are
// equal and at most 16 (elsewhere the prefetch registers would spill): one workgroup per CU walks a contiguous run of
// (column tile, batch item) work items -- batch-minor, so consecutive items
// share their spectrum lines -- and loads the next item's input while it
// transforms the current one.  No access needs a guard; the tables are
// boxed (lifted table loads would spill next to the prefetch).
// CONJ (the adjoint's conjugated spectrum) is a template parameter: as a
// runtime flag the compiler forms both products and selects, 6% of the
// kernel's VALU instructions.
// One FP32 complex value through a buffer resource: vo per lane, so uniform
// (bytes); AUX the cache policy (2: non-temporal).
using u32x2 = __attribute__((ext_vector_type(2))) unsigned;
template <typename T, int AUX>
__device__ __forceinline__ cx<T> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  static_assert(sizeof(cx<T>) == 8, "one FP32 complex value");
  return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX));
}
template <typename T, int AUX>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, cx<T> v) {
  static_assert(sizeof(cx<T>) == 8, "one FP32 complex value");
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, AUX);
}

template <typename T, class S, int C, bool CONJ>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, true>())) void k_rs_cols_persist(
    cx<T>* W, int64_t bstride, int n_valid, TableBox<T> Sq_, int nb, int items, int per, TableBox<T> tw_) {
  static_assert(sizeof(cx<T>) == 8, "buffer accesses of one FP32 complex value");
  const cx<T>* Sq = Sq_.p;
  constexpr int LS = line_stride<S, C, true>();
  __shared__ cx<T> smem[C * LS];
  const cx<T>* tw = tw_.p;
  using HI = HalfIn<S>;
  using HO = HalfOut<S>;
  constexpr int My = S::n, RIN = HI::R;
  constexpr uint32_t ES = sizeof(cx<T>);
  const int chunk = xcd_remap(blockIdx.x, gridDim.x);
  const int first = chunk * per, last = min(first + per, items);
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  cx<T>* lds = smem + c * LS;
  // A work item's columns kx = k0 + c (k0 = tile C) lie in 4-column tiles
  // k0 / 4 .. (k0 + C - 1) / 4 of the workspace and of the spectrum table.
  // Each is reached through a buffer resource whose base, the first of those
  // tiles, is uniform; a lane adds a 32-bit offset, and the row offset of
  // each register goes to the scalar offset, so no access needs 64-bit
  // address arithmetic.
  const int q = My / 2 + 1;
  struct Item {
    __amdgpu_buffer_rsrc_t w, sq;
    uint32_t lane;  // the lane's column within the tile run, in elements
  };
  auto item = [&](int id) -> Item {
    const int tile = id / nb, b = id - tile * nb;
    const int k0 = tile * C, ka = (k0 & 3) + c;
    const int ntiles = ((k0 & 3) + C + 3) / 4;
    Item it;
    it.w = __builtin_amdgcn_make_buffer_rsrc(W + b * bstride + (int64_t)(k0 >> 2) * n_valid * kTile, 0,
                                             (int)((uint32_t)ntiles * n_valid * kTile * ES), 0x00020000);
    it.sq = __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(Sq) + (int64_t)(k0 >> 2) * q * 4, 0,
                                              (int)((uint32_t)ntiles * q * 4 * ES), 0x00020000);
    it.lane = (uint32_t)(ka >> 2);
    it.lane = it.lane * (uint32_t)n_valid * kTile + (uint32_t)(ka & 3);
    return it;
  };
  // the lane's spectrum offset: the table holds 4-column tiles of q rows
  auto sq_lane = [&](int id) -> uint32_t {
    const int ka = ((id / nb) * C & 3) + c;
    return (uint32_t)(ka >> 2) * (uint32_t)q * 4 + (uint32_t)(ka & 3);
  };
  // threads j >= n/R0 exist when a later radix is smaller than the first;
  // they take no part in the first stage and load nothing
  const bool loader = HI::loads(j);
  cx<T> nxt[RIN];
  if (loader && first < last) {
    const Item it = item(first);
    const uint32_t vo = (it.lane + (uint32_t)j * kTile) * ES;
#pragma unroll
    for (int r = 0; r < RIN; ++r) nxt[r] = buf_load<T, 2>(it.w, vo, (uint32_t)(HI::index(j, r) - j) * kTile * ES);
  }
  for (int id = first; id < last; ++id) {
    cx<T> cur[RIN];
#pragma unroll
    for (int r = 0; r < RIN; ++r) cur[r] = nxt[r];
    if (loader && id + 1 < last) {
      const Item it = item(id + 1);
      const uint32_t vo = (it.lane + (uint32_t)j * kTile) * ES;
#pragma unroll
      for (int r = 0; r < RIN; ++r) nxt[r] = buf_load<T, 2>(it.w, vo, (uint32_t)(HI::index(j, r) - j) * kTile * ES);
    }
    const Item it = item(id);
    const uint32_t vs = sq_lane(id) * ES;
    const uint32_t vw = (it.lane + (uint32_t)j * kTile) * ES;
    // the first stage asks for i = HI::index(j, r): register r of cur
    auto load = [&](int i) -> cx<T> { return cur[(i - j) / HI::nr]; };
    auto mult = [&](int i, cx<T> v) -> cx<T> {
      const cx<T> h = buf_load<T, 0>(it.sq, vs + (uint32_t)min(i, My - i) * 4 * ES, 0);
      return CONJ ? cmulc(v, h) : cmul(v, h);
    };
    // the last stage stores i = HO::index(j, r) = j + r n / RL
    auto store = [&](int i, cx<T> v) {
      buf_store<T, 2>(it.w, vw, (uint32_t)(i - j) * kTile * ES, v);
    };
    static_assert(HO::index(1, 1) - 1 == HO::nr, "stores at j + r n / RL");
    conv_line<T, S, true, true>(lds, tw, j, load, mult, store);
  }
}

template <typename T, class S>
constexpr bool cols_persistent() {
  return tw_per_thread<T>() && conv_in_registers<S>() && S::rad[0] <= 16;
}

template <typename T, class S, int C>
hipError_t launch_rs_cols_c(cx<T>* W, int64_t bstride, int ncols, int n_valid, const cx<T>* Sq, int Mx, bool conj_spec,
                            int batch, const cx<T>* tw, hipStream_t s) {
  const int tiles = (ncols + C - 1) / C;
  constexpr bool can_half = S::rad[0] % 2 == 0 && S::rad[S::nst - 1] % 2 == 0;
  if constexpr (can_half) {
    if (2 * n_valid == S::n && ncols % C == 0) {
      if constexpr (cols_persistent<T, S>()) {
        // one workgroup per CU (the LDS footprint allows no more), each a
        // contiguous run of `per` items
        const int items = tiles * batch;
        const PersistSplit sp = persist_split(items, cu_count());
        if (conj_spec)
          hipLaunchKernelGGL((k_rs_cols_persist<T, S, C, true>), dim3(sp.groups), dim3(C * S::threads), 0, s, W,
                             bstride, n_valid, TableBox<T>{Sq}, batch, items, sp.per, TableBox<T>{tw});
        else
          hipLaunchKernelGGL((k_rs_cols_persist<T, S, C, false>), dim3(sp.groups), dim3(C * S::threads), 0, s, W,
                             bstride, n_valid, TableBox<T>{Sq}, batch, items, sp.per, TableBox<T>{tw});
      } else {
        hipLaunchKernelGGL((k_rs_cols<T, S, C, true, true>), dim3(tiles * batch), dim3(C * S::threads), 0, s, W,
                           bstride, ncols, n_valid, TableBox<T>{Sq}, Mx, conj_spec ? 1 : 0, tiles, TableBox<T>{tw});
      }
      return hipGetLastError();
    }
    if (2 * n_valid <= S::n) {
      hipLaunchKernelGGL((k_rs_cols<T, S, C, true>), dim3(tiles * batch), dim3(C * S::threads), 0, s, W, bstride,
                         ncols, n_valid, Sq, Mx, conj_spec ? 1 : 0, tiles, tw);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_rs_cols<T, S, C, false>), dim3(tiles * batch), dim3(C * S::threads), 0, s, W, bstride,
                     ncols, n_valid, Sq, Mx, conj_spec ? 1 : 0, tiles, tw);
  return hipGetLastError();
}

// Untuned choice among the bit-identical lines-per-workgroup variants of a
// non-persistent RS column pass: halve the lines (variant 1, then 2) while
// the pass has fewer than two workgroups per CU, so that small batch-1
// passes fill the chip.  Measured at batch 1 by the autotuner: 1024 points
// 10.7 -> 7.4 us (8 -> 2 lines), 1536 points 18.8 -> 11.3 us (4 -> 2
// lines).  The persistent pass keeps variant 0.
template <typename T, class S>
int rs_cols_fill_variant_s(int ncols, int n_valid, int batch) {
  using CF = Cfg<T, S, true>;
  if constexpr (!CF::fits) {
    return 0;
  } else {
    constexpr int C0 = CF::C, C1 = variant_lines<S, C0>(1), C2 = variant_lines<S, C0>(2);
    if constexpr (cols_persistent<T, S>()) {
      if (2 * n_valid == S::n && ncols % C0 == 0) return 0;
    }
    const int64_t want = 2 * (int64_t)cu_count();
    auto groups = [&](int c) { return (int64_t)((ncols + c - 1) / c) * batch; };
    if (C1 >= C0 || groups(C0) >= want) return 0;
    if (C2 >= C1 || groups(C1) >= want) return 1;
    return 2;
  }
}

template <typename T>
int rs_cols_fill_variant(int My, int ncols, int n_valid, int batch) {
  switch (My) {
#define LP_CASE(N, ...) \
  case N: return rs_cols_fill_variant_s<T, SchedOf<T, Sched<__VA_ARGS__>>>(ncols, n_valid, batch);
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return 0;
  }
}

template <typename T, class S>
hipError_t launch_rs_cols_s(cx<T>* W, int64_t bstride, int ncols, int n_valid, const cx<T>* Sq, int Mx, bool conj_spec,
                            int batch, const cx<T>* tw, hipStream_t s, int variant) {
  using CF = Cfg<T, S, true>;
  if constexpr (!CF::fits) {
    return hipErrorInvalidValue;
  } else {
    constexpr int C1 = variant_lines<S, CF::C>(1), C2 = variant_lines<S, CF::C>(2);
    if (variant == 1) return launch_rs_cols_c<T, S, C1>(W, bstride, ncols, n_valid, Sq, Mx, conj_spec, batch, tw, s);
    if (variant == 2) return launch_rs_cols_c<T, S, C2>(W, bstride, ncols, n_valid, Sq, Mx, conj_spec, batch, tw, s);
    return launch_rs_cols_c<T, S, CF::C>(W, bstride, ncols, n_valid, Sq, Mx, conj_spec, batch, tw, s);
  }
}

template <typename T>
hipError_t launch_rs_cols(int My, cx<T>* W, int64_t bstride, int ncols, int n_valid, const cx<T>* Sq, int Mx,
                          bool conj_spec, int batch, const cx<T>* tw, hipStream_t s, int variant) {
  if (batch <= 0 || ncols <= 0) return hipSuccess;
  switch (My) {
#define LP_CASE(N, ...)                                                                                        \
  case N: {                                                                                                    \
    if constexpr (has_alt<T, N>()) {                                                                           \
      if (variant >= kColVariants)                                                                             \
        return launch_rs_cols_s<T, typename AltSched<N>::type>(W, bstride, ncols, n_valid, Sq, Mx, conj_spec,  \
                                                               batch, tw, s, variant % kColVariants);          \
    }                                                                                                          \
    return launch_rs_cols_s<T, SchedOf<T, Sched<__VA_ARGS__>>>(W, bstride, ncols, n_valid, Sq, Mx, conj_spec,  \
                                                               batch, tw, s, variant % kColVariants);          \
  }
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// --------------------------------------------------- two-input mixing --
// out column = IFFT( ca Sa .* FFT(a) + cb Sb .* FFT(b) ) for the vectorial
// RS passes; Sa/Sb are half-table kernel spectra of the given parity
// kinds, ca/cb in {-1, +1}, optionally conjugated (adjoint).  `out` may be
// the same plane as `a` (in place per column).
template <typename T, class S, int C>
__global__ __launch_bounds__(2 * C * S::threads) void k_mix2_cols(
    const cx<T>* a, const cx<T>* bsrc, cx<T>* out, int64_t bstride, int ncols, int n_valid,
    const cx<T>* __restrict__ Sa, int kind_a, T ca, const cx<T>* __restrict__ Sb, int kind_b, T cb, int conj_spec,
    int Mx, int tiles, const cx<T>* __restrict__ tw) {
  constexpr int LE = line_stride<S, C, true>();
  __shared__ cx<T> smem[2 * C * LE];
  constexpr int My = S::n;
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int bt = id / tiles, tile = id - bt * tiles;
  // thread -> (input slot, column c, butterfly j)
  const int slot = threadIdx.x / (C * S::threads);
  const int t = threadIdx.x - slot * (C * S::threads);
  const int c = t % C, j = t / C;
  const int kx = tile * C + c;
  const bool valid = kx < ncols;
  cx<T>* lds = smem + (slot * C + c) * LE;
  const int64_t coff = bt * bstride + (int64_t)(kx >> kTileShift) * n_valid * kTile + (kx & (kTile - 1));
  const cx<T>* src = (slot == 0 ? a : bsrc) + coff;
  auto load = [&](int i) -> cx<T> {
    cx<T> v = czero<T>();
    if (valid && i < n_valid) v = src[i * kTile];
    return v;
  };
  auto st = [&](int i, cx<T> v) { lds[S::pad(i)] = v; };
  fft_line<T, -1, S>(lds, tw, j, load, st);
  // combine into slot 0 (each (c, k) owned by one thread)
  for (int e = threadIdx.x; e < C * My; e += 2 * C * S::threads) {
    const int cc = e % C, k = e / C;
    const int kxx = tile * C + cc;
    if (kxx >= ncols) continue;
    cx<T> ha = spec_at(Sa, kind_a, kxx, k, Mx, My);
    cx<T> hb = spec_at(Sb, kind_b, kxx, k, Mx, My);
    if (conj_spec) { ha.y = -ha.y; hb.y = -hb.y; }
    const int p = S::pad(k);
    const cx<T> va = smem[cc * LE + p], vb = smem[(C + cc) * LE + p];
    const cx<T> r = cadd(cscale(cmul(va, ha), ca), cscale(cmul(vb, hb), cb));
    smem[cc * LE + p] = r;
  }
  __syncthreads();
  // inverse transform of slot 0 by the slot-0 threads; slot-1 threads pass
  // an out-of-range butterfly index and only meet the barriers
  cx<T>* dst = out + coff;
  cx<T>* lds0 = smem + c * LE;
  auto load2 = [&](int i) -> cx<T> { return lds0[S::pad(i)]; };
  auto store = [&](int i, cx<T> v) {
    if (valid && i < n_valid) dst[i * kTile] = v;
  };
  fft_line<T, 1, S>(lds0, tw, slot == 0 ? j : S::threads, load2, store, true);
}

// Exact-half form (valid length n/2, column count a multiple of kTile; FP32
// schedules with the register hand-off): one column tile of kTile columns
// per workgroup, lanes of the columns interleaved, so every wave reads whole
// 32-byte tile rows (512 contiguous bytes); each column's threads transform a,
// then b (mix2_line), and run the one inverse transform.  The general form
// above gives each column its own pair of 256-thread slots with one column
// per workgroup, so its accesses are 8-byte segments.
template <typename T, class S>
constexpr bool mix2_exact_ok() {
  return tw_per_thread<T>() && conv_in_registers<S>() && S::threads * kTile <= kColThreads &&
         kTile * line_stride<S, kTile, true>() * (int)sizeof(cx<T>) <= kLdsBytes;
}

template <typename T, class S>
__global__ __launch_bounds__(kTile * S::threads, (waves_per_eu<T, S, kTile, true>())) void k_mix2_cols_x(
    const cx<T>* a, const cx<T>* bsrc, cx<T>* out, int64_t bstride, int n_valid, TableBox<T> Sa_, int kind_a, T ca,
    TableBox<T> Sb_, int kind_b, T cb, int conj_spec, int Mx, int tiles, TableBox<T> tw_) {
  constexpr int C = kTile;
  constexpr int LS = line_stride<S, C, true>();
  __shared__ cx<T> smem[C * LS];
  constexpr int My = S::n;
  const cx<T>* Sa = Sa_.p;
  const cx<T>* Sb = Sb_.p;
  // batch-minor order, as in the RS column pass
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int nb = gridDim.x / tiles;
  const int tile = id / nb, bt = id - tile * nb;
  const int c = (int)(threadIdx.x % C), j = (int)(threadIdx.x / C);
  const int kx = tile * C + c;
  cx<T>* lds = smem + c * LS;
  const int64_t coff = bt * bstride + (int64_t)tile * n_valid * kTile + c;
  const cx<T>* pa = a + coff;
  const cx<T>* pb = bsrc + coff;
  cx<T>* po = out + coff;
  auto load_a = [&](int i) -> cx<T> { return load_stream(&pa[i * kTile]); };
  auto load_b = [&](int i) -> cx<T> { return load_stream(&pb[i * kTile]); };
  auto mix = [&](int k, cx<T> va, cx<T> vb) -> cx<T> {
    cx<T> ha = spec_at(Sa, kind_a, kx, k, Mx, My), hb = spec_at(Sb, kind_b, kx, k, Mx, My);
    if (conj_spec) {
      ha.y = -ha.y;
      hb.y = -hb.y;
    }
    return cadd(cscale(cmul(va, ha), ca), cscale(cmul(vb, hb), cb));
  };
  auto store = [&](int i, cx<T> v) { store_stream(&po[i * kTile], v); };
  mix2_line<T, S>(lds, tw_.p, j, load_a, load_b, mix, store);
}

template <typename T, class S, int C>
hipError_t launch_mix2_cols_c(const cx<T>* a, const cx<T>* b, cx<T>* out, int64_t bstride, int ncols, int n_valid,
                              const cx<T>* Sa, int kind_a, T ca, const cx<T>* Sb, int kind_b, T cb, bool conj_spec,
                              int Mx, int batch, const cx<T>* tw, hipStream_t s) {
  const int tiles = (ncols + C - 1) / C;
  hipLaunchKernelGGL((k_mix2_cols<T, S, C>), dim3(tiles * batch), dim3(2 * C * S::threads), 0, s, a, b, out, bstride,
                     ncols, n_valid, Sa, kind_a, ca, Sb, kind_b, cb, conj_spec ? 1 : 0, Mx, tiles, tw);
  return hipGetLastError();
}

template <typename T, class S>
hipError_t launch_mix2_cols_s(const cx<T>* a, const cx<T>* b, cx<T>* out, int64_t bstride, int ncols, int n_valid,
                              const cx<T>* Sa, int kind_a, T ca, const cx<T>* Sb, int kind_b, T cb, bool conj_spec,
                              int Mx, int batch, const cx<T>* tw, hipStream_t s, int variant) {
  using CF = Cfg<T, S, true, 2, 512>;
  if constexpr (!CF::fits) {
    return hipErrorInvalidValue;
  } else {
    if constexpr (mix2_exact_ok<T, S>()) {
      if (variant == 0 && 2 * n_valid == S::n && ncols % kTile == 0) {
        const int tiles = ncols / kTile;
        hipLaunchKernelGGL((k_mix2_cols_x<T, S>), dim3(tiles * batch), dim3(kTile * S::threads), 0, s, a, b, out,
                           bstride, n_valid, TableBox<T>{Sa}, kind_a, ca, TableBox<T>{Sb}, kind_b, cb,
                           conj_spec ? 1 : 0, Mx, tiles, TableBox<T>{tw});
        return hipGetLastError();
      }
    }
    constexpr int C1 = variant_lines<S, CF::C>(1), C2 = variant_lines<S, CF::C>(2);
    if (variant == 1)
      return launch_mix2_cols_c<T, S, C1>(a, b, out, bstride, ncols, n_valid, Sa, kind_a, ca, Sb, kind_b, cb,
                                          conj_spec, Mx, batch, tw, s);
    if (variant == 2)
      return launch_mix2_cols_c<T, S, C2>(a, b, out, bstride, ncols, n_valid, Sa, kind_a, ca, Sb, kind_b, cb,
                                          conj_spec, Mx, batch, tw, s);
    return launch_mix2_cols_c<T, S, CF::C>(a, b, out, bstride, ncols, n_valid, Sa, kind_a, ca, Sb, kind_b, cb,
                                           conj_spec, Mx, batch, tw, s);
  }
}

template <typename T>
hipError_t launch_mix2_cols(int My, const cx<T>* a, const cx<T>* b, cx<T>* out, int64_t bstride, int ncols,
                            int n_valid, const cx<T>* Sa, int kind_a, T ca, const cx<T>* Sb, int kind_b,
                            T cb, bool conj_spec, int Mx, int batch, const cx<T>* tw, hipStream_t s, int variant) {
  if (batch <= 0 || ncols <= 0) return hipSuccess;
  switch (My) {
#define LP_CASE(N, ...)                                                                                             \
  case N:                                                                                                           \
    return launch_mix2_cols_s<T, SchedOf<T, Sched<__VA_ARGS__>>>(a, b, out, bstride, ncols, n_valid, Sa, kind_a, ca, Sb, \
                                                     kind_b, cb, conj_spec, Mx, batch, tw, s, variant);
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------- Bluestein --
// out[p] = post[p] * IFFT_L( FFT_L(pad(pre .* in)) .* chat )[p], p < n_out.
// Columns, and FP32 rows, run C lines per workgroup with the lanes of the
// lines interleaved (c = thread % C): the rows then share each stage's
// per-thread twiddle loads.  FP64 rows run one line per 256 threads.  The
// twiddle table is passed without __restrict__: with it the compiler treats
// the table loads as invariant, lifts every stage's loads ahead of the
// barriers and runs out of registers next to the chirp and filter loads.
template <typename T, bool COL>
constexpr bool bluestein_interleaved() {
  return COL || tw_per_thread<T>();
}

// Row lines of a Bluestein pass stream their input and output without cache
// retention (non-temporal) when the pass moves more than a cache could keep
// for the next pass anyway (128 MiB, half the MALL): the chirp and filter
// vectors, which every line reads, then stay cached (2048^2 at batch 8:
// rows 229.7 -> 223.3 us).  Smaller passes keep normal accesses, so that a
// following pass finds their output in the caches (the 96-setup plan lost
// 2% with streamed rows at batch 1).  Column lines are shared by
// neighbouring workgroups and never stream.
template <typename T>
inline bool bluestein_rows_streamed(bool col, int batch, int nlines, int n_in, int n_out) {
  const double bytes = (double)batch * nlines * (double)(n_in + n_out) * sizeof(cx<T>);
  return !col && bytes >= 128.0 * 1024 * 1024;
}

// PG = false: as for the row pass, an instance without the phase-gradient
// epilogue (used for row lines; the column instance measured no better).
// STAGE: the fused SLM stage of a plan setup (Slm) on the loads (first pass
// of a forward transform) or the stores (last pass of an adjoint); the
// field row and column of element i of line l follow from COL.
template <typename T, bool COL, class S, int C, bool HALF, bool EXACT = false, bool PG = true, bool STAGE = false>
__global__ __launch_bounds__(C * S::threads, (waves_per_eu<T, S, C, bluestein_interleaved<T, COL>(), 1,
                                                            HALF ? (bluestein_interleaved<T, COL>() ? 4 : 3) : 2>())) void k_bluestein(const cx<T>* in, cx<T>* out, Lines li, Lines lo,
                                                              int nlines, int n_in, int n_out,
                                                              const cx<T>* __restrict__ pre,
                                                              const cx<T>* __restrict__ chat,
                                                              const cx<T>* __restrict__ post, int tiles,
                                                              const cx<T>* tw, PhaseGrad<T> pg, Slm<T> st,
                                                              bool nt) {
  constexpr bool ILV = bluestein_interleaved<T, COL>();
  constexpr int LS = line_stride<S, C, ILV>();
  constexpr bool TL = !COL && ILV && conv_in_registers<S>() && tw_lds<T, S, C, ILV>();
  __shared__ cx<T> smem[C * LS + (TL ? TwLds<S>::elems : 0)];
  // (the first stage's barrier publishes the LDS twiddles before their use)
  tw = tw_source<TL, S>(smem + C * LS, tw, C * S::threads);
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int b = id / tiles, tile = id - b * tiles;
  const int c = ILV ? (int)(threadIdx.x % C) : (int)(threadIdx.x / S::threads);
  const int j = ILV ? (int)(threadIdx.x / C) : (int)(threadIdx.x % S::threads);
  const int l = tile * C + c;
  const bool valid = EXACT || l < nlines;
  cx<T>* lds = smem + c * LS;
  auto load = [&](int i) -> cx<T> {
    cx<T> v = czero<T>();
    if (valid && (EXACT || i < n_in)) {
      const int64_t io = line_off<COL>(li, b, l, i);
      v = cmul((COL || !nt) ? in[io] : load_stream(&in[io]), pre[i]);
      if constexpr (STAGE) {
        if (!st.adjoint) v = cmul(v, slm_factor(st, b, COL ? i : l, COL ? l : i));
      }
    }
    return v;
  };
  auto mult = [&](int i, cx<T> v) -> cx<T> { return cmul(v, chat[i]); };
  PhaseGradPre<T, S, PG && !STAGE && pg_preload<T, S, EXACT && HALF>()> pre_pg;
  pre_pg.load(pg, j, [&](int i) { return line_off<COL>(lo, b, l, i); });
  auto store = [&](int i, cx<T> v) {
    if (valid && (EXACT || i < n_out)) {
      const int64_t o = line_off<COL>(lo, b, l, i);
      const cx<T> g = cmul(v, post[i]);
      if constexpr (STAGE) {
        if (st.adjoint) {
          slm_adjoint_store(st, pg, out, b, COL ? i : l, COL ? l : i, o, g);
          return;
        }
      }
      if (out) {
        if (COL || !nt) out[o] = g;
        else store_stream(&out[o], g);
      }
      if constexpr (PG) {
        if (pg.grad) pre_pg.put(pg, i, j, o, g);
      }
    }
  };
  conv_line<T, S, HALF, HALF, TL>(lds, tw, j, load, mult, store);
}

template <typename T, bool COL, class S, int C, bool STAGE>
hipError_t launch_bluestein_c(const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in, int n_out,
                              const cx<T>* pre, const cx<T>* chat, const cx<T>* post, int batch, const cx<T>* tw,
                              hipStream_t s, PhaseGrad<T> pg, Slm<T> st) {
  const int tiles = (nlines + C - 1) / C;
  const bool nt = bluestein_rows_streamed<T>(COL, batch, nlines, n_in, n_out);
  constexpr bool can_half = S::rad[0] % 2 == 0 && S::rad[S::nst - 1] % 2 == 0;
  if constexpr (can_half) {
    if (2 * n_in == S::n && 2 * n_out == S::n && nlines % C == 0) {
      if (COL || pg.grad || STAGE)
        hipLaunchKernelGGL((k_bluestein<T, COL, S, C, true, true, true, STAGE>), dim3(tiles * batch),
                           dim3(C * S::threads), 0, s, in, out, li, lo, nlines, n_in, n_out, pre, chat, post, tiles, tw,
                           pg, st, nt);
      else
        hipLaunchKernelGGL((k_bluestein<T, COL, S, C, true, true, COL>), dim3(tiles * batch), dim3(C * S::threads),
                           0, s, in, out, li, lo, nlines, n_in, n_out, pre, chat, post, tiles, tw, pg, st, nt);
      return hipGetLastError();
    }
    if (2 * n_in <= S::n && 2 * n_out <= S::n) {
      hipLaunchKernelGGL((k_bluestein<T, COL, S, C, true, false, true, STAGE>), dim3(tiles * batch),
                         dim3(C * S::threads), 0, s, in, out, li, lo, nlines, n_in, n_out, pre, chat, post, tiles, tw,
                         pg, st, nt);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_bluestein<T, COL, S, C, false, false, true, STAGE>), dim3(tiles * batch),
                     dim3(C * S::threads), 0, s, in, out, li, lo, nlines, n_in, n_out, pre, chat, post, tiles, tw, pg,
                     st, nt);
  return hipGetLastError();
}

template <typename T, bool COL, class S, int C>
hipError_t launch_bluestein_cs(const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in, int n_out,
                               const cx<T>* pre, const cx<T>* chat, const cx<T>* post, int batch, const cx<T>* tw,
                               hipStream_t s, PhaseGrad<T> pg, const Slm<T>* slm) {
  if (slm && slm->active())
    return launch_bluestein_c<T, COL, S, C, true>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post, batch, tw, s,
                                                  pg, *slm);
  return launch_bluestein_c<T, COL, S, C, false>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post, batch, tw, s,
                                                 pg, Slm<T>{});
}

template <typename T, bool COL, class S>
hipError_t launch_bluestein_s(const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in, int n_out,
                              const cx<T>* pre, const cx<T>* chat, const cx<T>* post, int batch, const cx<T>* tw,
                              hipStream_t s, int variant, PhaseGrad<T> pg, const Slm<T>* slm) {
  // interleaved lines: up to 1024 threads per workgroup (for columns more
  // adjacent columns per row segment); FP64 rows: 512
  constexpr bool ILV = bluestein_interleaved<T, COL>();
  using CF = Cfg<T, S, ILV, 1, (ILV ? 1024 : 512)>;
  if constexpr (!CF::fits) {
    return hipErrorInvalidValue;
  } else {
    // the tuned column variants exist without the fused SLM stage only
    if constexpr (COL) {
      constexpr int C1 = variant_lines<S, CF::C>(1), C2 = variant_lines<S, CF::C>(2);
      if (!(slm && slm->active())) {
        if (variant == 1)
          return launch_bluestein_c<T, COL, S, C1, false>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post,
                                                          batch, tw, s, pg, Slm<T>{});
        if (variant == 2)
          return launch_bluestein_c<T, COL, S, C2, false>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post,
                                                          batch, tw, s, pg, Slm<T>{});
      }
    }
    constexpr int C = (ILV && !COL) ? row_lines_two_per_cu<T, S, CF::C>() : CF::C;
    return launch_bluestein_cs<T, COL, S, C>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post, batch, tw, s, pg,
                                             slm);
  }
}

template <typename T>
hipError_t launch_bluestein(int L, bool col, const cx<T>* in, cx<T>* out, Lines li, Lines lo, int nlines, int n_in,
                            int n_out, const cx<T>* pre, const cx<T>* chat, const cx<T>* post, int batch,
                            const cx<T>* tw, hipStream_t s, int variant, const cx<T>* pg_u, T* pg_grad, int pg_acc,
                            const Slm<T>* slm) {
  if (nlines <= 0 || batch <= 0) return hipSuccess;
  PhaseGrad<T> pg;
  pg.u = pg_u;
  pg.grad = pg_grad;
  pg.acc = pg_acc;
  switch (L) {
#define LP_CASE(N, ...)                                                                                             \
  case N: {                                                                                                         \
    if constexpr (has_alt<T, N>()) {                                                                                \
      using A = typename AltSched<N>::type;                                                                         \
      if (variant >= kColVariants)                                                                                  \
        return col ? launch_bluestein_s<T, true, A>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post, batch,  \
                                                    tw, s, variant % kColVariants, pg, slm)                         \
                   : launch_bluestein_s<T, false, A>(in, out, li, lo, nlines, n_in, n_out, pre, chat, post, batch, \
                                                     tw, s, 0, pg, slm);                                            \
    }                                                                                                               \
    return col ? launch_bluestein_s<T, true, SchedOf<T, Sched<__VA_ARGS__>>>(in, out, li, lo, nlines, n_in, n_out,  \
                                                                           pre, chat, post, batch, tw, s,           \
                                                                           variant % kColVariants, pg, slm)         \
               : launch_bluestein_s<T, false, SchedOf<T, Sched<__VA_ARGS__>>>(in, out, li, lo, nlines, n_in, n_out, \
                                                                            pre, chat, post, batch, tw, s, 0, pg,   \
                                                                            slm);                                   \
  }
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Lines per workgroup of a tuner candidate (kind 0: RS column pass, 1:
// vectorial mixing, 2: Bluestein columns, 3: Bluestein rows) at length n,
// 0 if unsupported.  Candidates v < kColVariants run the built-in schedule
// with C >> v lines (rows: v = 0 only); v + kColVariants the same on the
// length's alternative schedule (RS columns and Bluestein passes, FP32).
template <typename T, class S>
int candidate_lines(int kind, int v) {
  constexpr int c0 = Cfg<T, S, true>::C, c1 = Cfg<T, S, true, 2, 512>::C, c2 = Cfg<T, S, true, 1, 1024>::C;
  if (kind == 3) {
    if (v != 0) return 0;
    constexpr bool ILV = bluestein_interleaved<T, false>();
    using CF = Cfg<T, S, ILV, 1, (ILV ? 1024 : 512)>;
    return (ILV ? row_lines_two_per_cu<T, S, CF::C>() : CF::C);
  }
  const int c = kind == 0 ? c0 : (kind == 1 ? c1 : c2);
  return S::n >= kTuneMinLength ? cmax(1, c >> v) : c;
}

template <typename T>
int col_pass_lines(int kind, int n, int variant) {
  if (variant < 0 || variant >= kColVariants * kSchedVariants || kind < 0 || kind > 3) return 0;
  const int v = variant % kColVariants;
  const bool alt = variant >= kColVariants;
  if (alt && kind == 1) return 0;  // vectorial mixing: built-in schedule only
  switch (n) {
#define LP_CASE(N, ...)                                                                             \
  case N: {                                                                                         \
    if (alt) {                                                                                      \
      if constexpr (has_alt<T, N>()) return candidate_lines<T, typename AltSched<N>::type>(kind, v); \
      return 0;                                                                                     \
    }                                                                                               \
    return candidate_lines<T, SchedOf<T, Sched<__VA_ARGS__>>>(kind, v);                             \
  }
    LP_LENGTHS(LP_CASE)
#undef LP_CASE
    default:
      return 0;
  }
}

}  // namespace lp
