// Device-side mixed-radix (2/3) FFT engine for CDNA4 (gfx950).
//
// A "line" is one 1-D transform of length n = 2^a 3^b <= 8192 handled by T
// threads of a workgroup.  The transform is a Stockham autosort sequence of
// stages with radices R_s (prod R_s = n).  In stage s every active thread
// owns one radix-R_s butterfly: it reads R values at stride n/R_s, applies
// the stage twiddles, runs an in-register DFT_R and writes R values.  The
// first stage reads through a caller-supplied load functor (global memory,
// zero padding and pre-multiplication fused in), intermediate stages go
// through LDS, and the last stage hands natural-order outputs to a store
// functor (global memory with cropping/post-multiplication, or LDS for a
// following transform).  The twiddle table holds, for stage s, the values
// W_{Ns R}^{r k} (r < R, k < Ns): for FP64 at tw[off_s + (r-1) Ns + k], so
// lanes with consecutive k read consecutive entries; for FP32 as one run per
// thread, tw[off_s + k R + r] (Sched::twoff).  FP32 row passes may read them
// from small LDS tables instead (TwLds).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "lengths.hpp"

namespace lp {

// ---------------------------------------------------------------- complex --
// Interleaved (re, im) pair: the layout of torch.complex64 / complex128.
template <typename T> struct alignas(2 * sizeof(T)) cx { T x, y; };

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  V r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
template <typename V> __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { a.x *= s; a.y *= s; return a; }
// multiply by -i (DIR<0) or +i (DIR>0)
template <int DIR, typename V> __device__ __forceinline__ V mul_i(V a) {
  V r;
  if (DIR < 0) { r.x = a.y; r.y = -a.x; } else { r.x = -a.y; r.y = a.x; }
  return r;
}

// ------------------------------------------- compile-time sin/cos of 2 pi p/q
struct CS { double c, s; };
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int n = 1; n < 14; ++n) { t *= -x * x / double((2 * n) * (2 * n + 1)); s += t; }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 14; ++n) { t *= -x * x / double((2 * n - 1) * (2 * n)); s += t; }
  return s;
}
// exact octant reduction in integers, Taylor on [0, pi/4]
constexpr CS sincos2pi(long p, long q) {
  p %= q;
  if (p < 0) p += q;
  const long quad = (4 * p) / q;
  long rem = 4 * p - quad * q;  // angle within quadrant = (pi/2) rem / q
  bool swap = false;
  if (2 * rem > q) { rem = q - rem; swap = true; }
  const double x = 1.5707963267948966192313216916398 * double(rem) / double(q);
  double c = taylor_cos(x), s = taylor_sin(x);
  if (swap) { double t = c; c = s; s = t; }
  double rc = c, rs = s;
  if (quad == 1) { rc = -s; rs = c; }
  else if (quad == 2) { rc = -c; rs = -s; }
  else if (quad == 3) { rc = s; rs = -c; }
  return CS{rc, rs};
}

// multiply by the constant W_R^M in direction DIR (exp(DIR * 2 pi i M / R));
// M is a template parameter so that every constant folds at compile time
template <int R, int DIR, int M, typename T>
__device__ __forceinline__ cx<T> mul_const(cx<T> a) {
  using V = cx<T>;
  constexpr int mm = ((M % R) + R) % R;
  constexpr CS w = sincos2pi(mm, R);
  constexpr double c = w.c;
  constexpr double s = DIR * w.s;
  if constexpr (mm == 0) {
    return a;
  } else if constexpr (4 * mm == R) {
    return mul_i<DIR>(a);
  } else if constexpr (2 * mm == R) {
    a.x = -a.x;
    a.y = -a.y;
    return a;
  } else if constexpr (4 * mm == 3 * R) {
    return mul_i<-DIR>(a);
  } else if constexpr (8 * mm == R || 8 * mm == 3 * R || 8 * mm == 5 * R || 8 * mm == 7 * R) {
    // |c| == |s| == 1/sqrt 2
    constexpr T h = T(c > 0 ? c : -c);
    constexpr T sc = T(c > 0 ? 1 : -1), ss = T(s > 0 ? 1 : -1);
    V r;
    const T re = sc * a.x - ss * a.y;
    const T im = ss * a.x + sc * a.y;
    r.x = re * h;
    r.y = im * h;
    return r;
  } else {
    constexpr T cc = T(c), sv = T(s);
    V r;
    r.x = a.x * cc - a.y * sv;
    r.y = a.x * sv + a.y * cc;
    return r;
  }
}

// ------------------------------------------------------- in-register DFTs --
// Dft<R, DIR>: v[k] <- sum_r v[r] exp(DIR 2 pi i r k / R), natural order.
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<1, DIR> {
  template <typename T> __device__ __forceinline__ static void run(cx<T>*) {}
};
template <int DIR> struct Dft<2, DIR> {
  template <typename T> __device__ __forceinline__ static void run(cx<T>* v) {
    using V = cx<T>;
    V a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};
template <int DIR> struct Dft<3, DIR> {
  template <typename T> __device__ __forceinline__ static void run(cx<T>* v) {
    using V = cx<T>;
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    V t = cadd(v[1], v[2]);
    V d = csub(v[1], v[2]);
    V m; m.x = v[0].x - T(0.5) * t.x; m.y = v[0].y - T(0.5) * t.y;
    v[0] = cadd(v[0], t);
    // DIR * i * (sqrt3/2) * d
    V s = mul_i<DIR>(d); s.x *= h; s.y *= h;
    v[1] = cadd(m, s);
    v[2] = csub(m, s);
  }
};
template <int DIR> struct Dft<4, DIR> {
  template <typename T> __device__ __forceinline__ static void run(cx<T>* v) {
    using V = cx<T>;
    V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    V t2 = cadd(v[1], v[3]), t3 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
  }
};

template <int R> struct FirstFactor {
  static constexpr int value = (R % 4 == 0 && R != 4) ? 4 : (R % 3 == 0 && R != 3) ? 3 : (R % 2 == 0 && R != 2) ? 2 : R;
};

// y[I] *= W_R^{(I / B) (I % B)} for all I < R
template <int R, int B, int DIR, typename T, int... I>
__device__ __forceinline__ void twiddle_block(cx<T>* y, std::integer_sequence<int, I...>) {
  ((y[I] = mul_const<R, DIR, (I / B) * (I % B), T>(y[I])), ...);
}

// Composite R = A B: r = r1 + A r2, k = k2 + B k1.
template <int R, int DIR> struct Dft {
  static constexpr int A = FirstFactor<R>::value;
  static constexpr int B = R / A;
  template <typename T> __device__ __forceinline__ static void run(cx<T>* v) {
    using V = cx<T>;
    V y[R];
#pragma unroll
    for (int r1 = 0; r1 < A; ++r1) {
      V t[B];
#pragma unroll
      for (int r2 = 0; r2 < B; ++r2) t[r2] = v[r1 + A * r2];
      Dft<B, DIR>::template run<T>(t);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) y[r1 * B + k2] = t[k2];
    }
    twiddle_block<R, B, DIR, T>(y, std::make_integer_sequence<int, R>{});
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      V t[A];
#pragma unroll
      for (int r1 = 0; r1 < A; ++r1) t[r1] = y[r1 * B + k2];
      Dft<A, DIR>::template run<T>(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) v[k2 + B * k1] = t[k1];
    }
  }
};

// ------------------------------------------------------- radix schedules --
// The supported lengths and their schedules: LP_LENGTHS (lengths.hpp).
constexpr int kMaxStages = 4;

// Twiddle table layout of an element type (see Sched::twoff).
template <typename T>
__host__ __device__ constexpr bool tw_per_thread() {
  return sizeof(T) == 4;
}

template <int... Rs> struct Sched {
  static constexpr int nst = sizeof...(Rs);
  static constexpr int rad[nst] = {Rs...};
  static constexpr int n = (1 * ... * Rs);
  static constexpr int rmin() {
    int m = rad[0];
    for (int i = 1; i < nst; ++i) m = rad[i] < m ? rad[i] : m;
    return m;
  }
  static constexpr int threads = n / rmin();
  static constexpr int ns(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= rad[i];
    return p;
  }
  // Offset of stage s in the twiddle table, for two layouts of W_{Ns R}^{r k}
  // (r = 0..R-1, k = 0..Ns-1) chosen by element type:
  //  * per thread (FP32): off + k R + r, with r = 0 (the value 1) stored, so
  //    a thread's R twiddles are one aligned run of memory: fewer and wider
  //    loads from one base address;
  //  * per stage (FP64): off + (r - 1) Ns + k, so the lanes' consecutive k
  //    read consecutive 16-byte values (the wider loads do not pay there).
  static constexpr int twoff(int s, bool per_thread) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += (per_thread ? rad[i] : rad[i] - 1) * ns(i);
    return off;
  }
  static constexpr int twsize(bool per_thread) { return nst > 1 ? twoff(nst, per_thread) : 1; }
  // LDS padding: one element per 2^pad_shift.  With the first radix R0 a
  // power of two, shift log2(R0) turns the first stage's stride-R0 scatter
  // into an odd stride (R0 + 1), so a half-wave's writes hit distinct banks.
  static constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
  static constexpr bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
  static constexpr int pad_shift = (pow2(rad[0]) && rad[0] >= 4) ? ilog2(rad[0]) : 5;
  static constexpr int line_elems = n + (n >> pad_shift) + 1;
  __host__ __device__ static constexpr int pad(int i) { return i + (i >> pad_shift); }
  // pad(m R + r) == pad(m R) + r for 0 <= r < R when R divides 2^pad_shift
  static constexpr bool contiguous_pad(int R) { return ((1 << pad_shift) % R) == 0; }
  // pad(b + r m) == pad(b) + r pstride(m) when 2^pad_shift divides m: the
  // strided accesses of a stage become one base plus immediate offsets
  static constexpr bool stride_pad(int m) { return m % (1 << pad_shift) == 0; }
  static constexpr int pstride(int m) { return m + (m >> pad_shift); }
};


// The schedule that element type T runs for a table entry S.  At 2048 the
// table holds 16*8*16, whose equal first and last radices let the FP32
// convolutions keep the spectrum product in registers (1024^2 grids: RS
// column pass 160 -> 129 us, Bluestein rows 102 -> 92 us at batch 8).  FP64
// keeps 16*16*8: with four lines per workgroup its 16-point stages spill.
template <typename T, class S> struct SchedFor { using type = S; };
template <> struct SchedFor<double, Sched<16, 8, 16>> { using type = Sched<16, 16, 8>; };
template <typename T, class S> using SchedOf = typename SchedFor<T, S>::type;

// The alternative schedule of length N (LP_ALT_LENGTHS), or void.
template <int N> struct AltSched { using type = void; };
#define LP_ALT_DEF(N, ...) \
  template <> struct AltSched<N> { using type = Sched<__VA_ARGS__>; };
LP_ALT_LENGTHS(LP_ALT_DEF)
#undef LP_ALT_DEF
// Element type T may run the alternative schedule of length N.
template <typename T, int N>
constexpr bool has_alt() {
  return sizeof(T) == 4 && !std::is_void<typename AltSched<N>::type>::value;
}

// Inputs of the first stage of a half-input transform: thread j < n/R0
// reads elements j + r n/R0 for r < R0/2, which cover [0, n/2) once each.
// Persistent passes prefetch exactly these elements.
template <class S> struct HalfIn {
  static constexpr int nr = S::n / S::rad[0], R = S::rad[0] / 2;
  __host__ __device__ static constexpr bool loads(int j) { return j < nr; }
  __host__ __device__ static constexpr int index(int j, int r) { return j + r * nr; }
};
// Outputs of the last stage of a half-output transform: thread j < n/RL
// stores elements j + r n/RL for r < RL/2, covering [0, n/2) once each.
template <class S> struct HalfOut {
  static constexpr int RL = S::rad[S::nst - 1];
  static constexpr int nr = S::n / RL, R = RL / 2;
  __host__ __device__ static constexpr bool stores(int j) { return j < nr; }
  __host__ __device__ static constexpr int index(int j, int r) { return j + r * nr; }
};

// FP32 twiddles from LDS tables, for schedules of two or three stages
// R0 R1 (R2).  The first twiddled stage (Ns = R0) reads T1[r][k] =
// W_{R0 R1}^{k r} (k < R0, r < R1) directly.  The second (Ns = R0 R1, three
// stages) forms W_n^{k r} = W_{R1 R2}^{a r} W_n^{b r} with k = R0 a + b from
// Thi[r][a] (a < R1, r < R2) and Tlo[r][b] (b < R0): one complex product of
// two correctly rounded values.  When R0 = R1 = R2, Thi is T1 and is stored
// once (16*16*16: 512 entries, 4 KiB).  Lanes with consecutive k read
// consecutive entries.  A kernel using them fills the tables once per
// workgroup (fill) and passes their LDS address in place of the global table,
// with the engine's TL flag set.
template <class S>
struct TwLds {
  static constexpr bool ok = S::nst == 2 || S::nst == 3;
  static constexpr int R0 = S::rad[0], R1 = ok ? S::rad[1] : 1, R2 = S::nst == 3 ? S::rad[2] : 1;
  static constexpr bool shared_hi = S::nst == 3 && R0 == R1 && R1 == R2;
  static constexpr int o_hi = shared_hi ? 0 : R0 * R1;
  static constexpr int o_lo = shared_hi ? R0 * R1 : R0 * R1 + R1 * R2;
  static constexpr int elems = S::nst == 3 ? o_lo + R0 * R2 : R0 * R1;
  // LDS entry of the first twiddled stage's W^{k r}; the two entries whose
  // product is the second's
  __host__ __device__ static constexpr int at1(int k, int r) { return r * R0 + k; }
  __host__ __device__ static constexpr int at2_hi(int k, int r) { return o_hi + r * R1 + k / R0; }
  __host__ __device__ static constexpr int at2_lo(int k, int r) { return o_lo + r * R0 + k % R0; }
  // the global per-thread FP32 table entry (stage 1 at k R1 + r, stage 2 at
  // R0 R1 + k R2 + r) that LDS entry e copies
  __host__ __device__ static constexpr int src(int e) {
    return e < R0 * R1 ? (e % R0) * R1 + e / R0
           : e < o_lo  ? R0 * R1 + R0 * ((e - R0 * R1) % R1) * R2 + (e - R0 * R1) / R1
                       : R0 * R1 + ((e - o_lo) % R0) * R2 + (e - o_lo) / R0;
  }
  template <int s>
  __device__ __forceinline__ static cx<float> get(const cx<float>* tl, int k, int r) {
    static_assert(s == 1 || (s == 2 && S::nst == 3), "twiddled stages of two- and three-stage schedules");
    if constexpr (s == 1) return tl[at1(k, r)];
    else return cmul(tl[at2_hi(k, r)], tl[at2_lo(k, r)]);
  }
  // every thread of the workgroup calls this; the caller synchronises before use
  __device__ __forceinline__ static void fill(cx<float>* tl, const cx<float>* tw, int tid, int nthreads) {
    for (int e = tid; e < elems; e += nthreads) tl[e] = tw[src(e)];
  }
};

// HALF_IN: inputs with index >= n/2 are zero (skipped at compile time);
// HALF_OUT: only outputs with index < n/2 are consumed (the rest is never
// computed).  Both need an even first (last) radix.
// TL: tw is the LDS twiddle tables of TwLds<S> (FP32, two or three stages).
template <typename T, int DIR, class S, int s, bool HALF_IN, bool HALF_OUT, bool TL, class Load, class Store>
__device__ __forceinline__ void ct_stage(cx<T>* __restrict__ lds, const cx<T>* __restrict__ tw, int j,
                                         bool sync_first, Load& load, Store& store) {
  using V = cx<T>;
  constexpr int R = S::rad[s];
  constexpr int nr = S::n / R;
  constexpr int Ns = S::ns(s);
  constexpr bool first = s == 0, last = s == S::nst - 1;
  constexpr int r_in = (first && HALF_IN) ? R / 2 : R;
  constexpr int r_out = (last && HALF_OUT) ? R / 2 : R;
  static_assert(!(first && HALF_IN) || R % 2 == 0, "half input needs an even first radix");
  static_assert(!(last && HALF_OUT) || R % 2 == 0, "half output needs an even last radix");
  const bool act = j < nr;
  V v[R];
  if (act) {
    if constexpr (first) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r < r_in) v[r] = load(j + r * nr);
        else v[r] = mk<T>(T(0), T(0));
      }
    } else if constexpr (S::stride_pad(nr)) {
      const cx<T>* p = lds + S::pad(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = p[r * S::pstride(nr)];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = lds[S::pad(j + r * nr)];
    }
  }
  if (!first || sync_first) __syncthreads();
  if (act) {
    const int k = j % Ns;
    const int q = j / Ns;
    if constexpr (!first && TL) {
      static_assert(std::is_same<T, float>::value && TwLds<S>::ok, "LDS twiddles: FP32, two or three stages");
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const V w = TwLds<S>::template get<s>(tw, k, r);
        v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
      }
    } else if constexpr (!first) {
      constexpr bool pt = tw_per_thread<T>();
      const V* t = tw + S::twoff(s, pt) + (pt ? k * R : k);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const V w = pt ? t[r] : t[(r - 1) * Ns];
        v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
      }
    }
    Dft<R, DIR>::template run<T>(v);
    if constexpr (last) {
#pragma unroll
      for (int r = 0; r < r_out; ++r) store(j + r * nr, v[r]);
    } else if constexpr (Ns > 1 && S::stride_pad(Ns)) {
      cx<T>* p = lds + S::pad(q * Ns * R + k);
#pragma unroll
      for (int r = 0; r < R; ++r) p[r * S::pstride(Ns)] = v[r];
    } else if constexpr (Ns == 1 && S::contiguous_pad(R)) {
      // first stage: outputs q R + r are contiguous after padding
      cx<T>* p = lds + S::pad(q * R);
#pragma unroll
      for (int r = 0; r < R; ++r) p[r] = v[r];
    } else {
      const int base = q * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[S::pad(base + r * Ns)] = v[r];
    }
  }
  __syncthreads();
}

template <typename T, int DIR, class S, bool HI, bool HO, bool TL, class Load, class Store, int... I>
__device__ __forceinline__ void ct_line_impl(cx<T>* lds, const cx<T>* tw, int j, bool sync_first, Load& load,
                                             Store& store, std::integer_sequence<int, I...>) {
  (ct_stage<T, DIR, S, I, HI, HO, TL>(lds, tw, j, sync_first, load, store), ...);
}

// One transform of one line of length S::n by threads j = 0..S::threads-1.
// Every thread of the workgroup must call this (barriers inside).
// DIR = -1: forward (exp(-2 pi i jk/n)); DIR = +1: inverse, unnormalised.
// load_reads_lds: the load functor reads this workgroup's LDS, so the first
// stage waits for every read before writing.
template <typename T, int DIR, class S, bool HALF_IN = false, bool HALF_OUT = false, bool TL = false, class Load,
          class Store>
__device__ __forceinline__ void fft_line(cx<T>* lds, const cx<T>* tw, int j, Load load, Store store,
                                         bool load_reads_lds = false) {
  ct_line_impl<T, DIR, S, HALF_IN, HALF_OUT, TL>(lds, tw, j, load_reads_lds, load, store,
                                                std::make_integer_sequence<int, S::nst>{});
}

// Forward transform, pointwise multiply, inverse transform of one line
// (the convolution core of the RS column pass and of Bluestein's method).
// When the first and last radices agree, the last forward stage and the
// first inverse stage touch the same indices j + r n/R in the same thread
// (Stockham order), so the product stays in registers: one LDS write, one
// LDS read and two barriers fewer than two separate fft_line calls.
// mult(i, v) returns the product for frequency i.
// The two halves of the register hand-off: conv_fwd_last reads the last
// forward stage's inputs from LDS and leaves its outputs, frequencies
// j + r n/R, in v; conv_inv_first runs the first inverse stage on v and
// writes its outputs to LDS.
template <typename T, class S, bool TL>
__device__ __forceinline__ void conv_fwd_last(cx<T>* __restrict__ lds, const cx<T>* __restrict__ tw, int j,
                                              cx<T> (&v)[S::rad[S::nst - 1]]) {
  using V = cx<T>;
  constexpr int sl = S::nst - 1;
  constexpr int R = S::rad[sl];
  constexpr int nr = S::n / R;
  static_assert(S::rad[0] == R && S::ns(sl) == nr, "register hand-off needs equal first and last radices");
  const bool act = j < nr;
  if (act) {
    if constexpr (S::stride_pad(nr)) {
      const cx<T>* p = lds + S::pad(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = p[r * S::pstride(nr)];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = lds[S::pad(j + r * nr)];
    }
  }
  __syncthreads();
  if (act) {
    if constexpr (TL) {
      static_assert(std::is_same<T, float>::value && TwLds<S>::ok, "LDS twiddles: FP32, two or three stages");
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], TwLds<S>::template get<sl>(tw, j, r));
    } else {
      constexpr bool pt = tw_per_thread<T>();
      const V* t = tw + S::twoff(sl, pt) + (pt ? j * R : j);
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], pt ? t[r] : t[(r - 1) * nr]);
    }
    Dft<R, -1>::template run<T>(v);
  }
}

template <typename T, class S>
__device__ __forceinline__ void conv_inv_first(cx<T>* __restrict__ lds, int j, cx<T> (&v)[S::rad[S::nst - 1]]) {
  constexpr int R = S::rad[S::nst - 1];
  constexpr int nr = S::n / R;
  if (j < nr) {
    Dft<R, 1>::template run<T>(v);
    // first inverse stage (Ns = 1): outputs j R + r
    if constexpr (S::contiguous_pad(R)) {
      cx<T>* p = lds + S::pad(j * R);
#pragma unroll
      for (int r = 0; r < R; ++r) p[r] = v[r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[S::pad(j * R + r)] = v[r];
    }
  }
  __syncthreads();
}

template <typename T, class S, bool TL, class Mult>
__device__ __forceinline__ void conv_mid_stage(cx<T>* __restrict__ lds, const cx<T>* __restrict__ tw, int j,
                                               Mult& mult) {
  constexpr int R = S::rad[S::nst - 1];
  constexpr int nr = S::n / R;
  cx<T> v[R];
  conv_fwd_last<T, S, TL>(lds, tw, j, v);
  if (j < nr) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = mult(j + r * nr, v[r]);
  }
  conv_inv_first<T, S>(lds, j, v);
}

template <typename T, class S, bool HI, bool HO, bool TL, class Load, class Mult, class Store, int... I>
__device__ __forceinline__ void conv_line_impl(cx<T>* lds, const cx<T>* tw, int j, bool sync_first, Load& load,
                                               Mult& mult, Store& store, std::integer_sequence<int, I...>) {
  auto none = [](int, cx<T>) {};
  (ct_stage<T, -1, S, I, HI, false, TL>(lds, tw, j, sync_first, load, none), ...);
  conv_mid_stage<T, S, TL>(lds, tw, j, mult);
  (ct_stage<T, 1, S, I + 1, false, HO, TL>(lds, tw, j, false, load, store), ...);
}

template <class S>
constexpr bool conv_in_registers() {
  return S::nst >= 2 && S::rad[0] == S::rad[S::nst - 1];
}

template <typename T, class S, bool HALF_IN = false, bool HALF_OUT = false, bool TL = false, class Load, class Mult,
          class Store>
__device__ __forceinline__ void conv_line(cx<T>* lds, const cx<T>* tw, int j, Load load, Mult mult, Store store,
                                          bool load_reads_lds = false) {
  if constexpr (conv_in_registers<S>()) {
    conv_line_impl<T, S, HALF_IN, HALF_OUT, TL>(lds, tw, j, load_reads_lds, load, mult, store,
                                                std::make_integer_sequence<int, S::nst - 1>{});
  } else {
    static_assert(!TL, "LDS twiddles: register hand-off schedules only");
    auto mid = [&](int i, cx<T> v) { lds[S::pad(i)] = mult(i, v); };
    fft_line<T, -1, S, HALF_IN, false>(lds, tw, j, load, mid, load_reads_lds);
    auto load2 = [&](int i) -> cx<T> { return lds[S::pad(i)]; };
    fft_line<T, 1, S, false, HALF_OUT>(lds, tw, j, load2, store, true);
  }
}

// Two-input convolution of one line: out = IFFT( mix(k, FFT(a)[k], FFT(b)[k]) )
// with zero upper input halves and the lower output half kept.  The same
// threads transform a and then b, holding FFT(a) in registers while b runs
// through the LDS stages; one inverse transform follows.  Needs the register
// hand-off (equal first and last radix).
template <typename T, class S, class LoadA, class LoadB, class Mix, class Store, int... I>
__device__ __forceinline__ void mix2_line_impl(cx<T>* lds, const cx<T>* tw, int j, LoadA& load_a, LoadB& load_b,
                                               Mix& mix, Store& store, std::integer_sequence<int, I...>) {
  constexpr int R = S::rad[S::nst - 1];
  constexpr int nr = S::n / R;
  auto none = [](int, cx<T>) {};
  cx<T> va[R], vb[R];
  (ct_stage<T, -1, S, I, true, false, false>(lds, tw, j, false, load_a, none), ...);
  conv_fwd_last<T, S, false>(lds, tw, j, va);
  (ct_stage<T, -1, S, I, true, false, false>(lds, tw, j, false, load_b, none), ...);
  conv_fwd_last<T, S, false>(lds, tw, j, vb);
  if (j < nr) {
#pragma unroll
    for (int r = 0; r < R; ++r) va[r] = mix(j + r * nr, va[r], vb[r]);
  }
  conv_inv_first<T, S>(lds, j, va);
  (ct_stage<T, 1, S, I + 1, false, true, false>(lds, tw, j, false, load_a, store), ...);
}

template <typename T, class S, class LoadA, class LoadB, class Mix, class Store>
__device__ __forceinline__ void mix2_line(cx<T>* lds, const cx<T>* tw, int j, LoadA load_a, LoadB load_b, Mix mix,
                                          Store store) {
  static_assert(conv_in_registers<S>(), "two-input convolution needs the register hand-off");
  mix2_line_impl<T, S>(lds, tw, j, load_a, load_b, mix, store, std::make_integer_sequence<int, S::nst - 1>{});
}

// Host-side description of a length's schedule (for twiddle tables).
struct SchedInfo {
  int n, nst, threads;
  int rad[kMaxStages];
};

template <class S>
inline void sched_fill(SchedInfo* out) {
  out->n = S::n;
  out->nst = S::nst;
  out->threads = S::threads;
  for (int i = 0; i < S::nst; ++i) out->rad[i] = S::rad[i];
}

// fp64: the schedule FP64 transforms run (SchedOf<double, ...>); alt: the
// alternative schedule (FP32 only; false if the length has none)
inline bool sched_info(int n, SchedInfo* out, bool fp64 = false, bool alt = false) {
  if (alt) {
    if (fp64) return false;
    switch (n) {
#define LP_ALT_CASE(N, ...)                    \
  case N:                                      \
    sched_fill<Sched<__VA_ARGS__>>(out);       \
    return true;
      LP_ALT_LENGTHS(LP_ALT_CASE)
#undef LP_ALT_CASE
      default:
        return false;
    }
  }
  switch (n) {
#define LP_SCHED_CASE(N, ...)                                                             \
  case N: {                                                                               \
    if (fp64) sched_fill<SchedOf<double, Sched<__VA_ARGS__>>>(out);                       \
    else sched_fill<Sched<__VA_ARGS__>>(out);                                             \
    return true;                                                                          \
  }
    LP_LENGTHS(LP_SCHED_CASE)
#undef LP_SCHED_CASE
    default:
      return false;
  }
}

}  // namespace lp
