// Device-side FFT building blocks for gfx950 (wave64, LDS exchange).
//
// A line of P complex points is transformed by TL = P/E threads that each
// hold E points in registers.  Thread t always holds points t + TL*q,
// q = 0..E-1, at the start of every stage.  Each stage is a Stockham
// autosort radix-R step (no bit reversal): butterfly b takes inputs
// x[b + i P/R], applies the twiddles exp(+-2 pi i * i*k/(Ns R)) with
// k = b mod Ns (Ns = product of the radices already done), a radix-R DFT in
// registers, and writes y[(b/Ns) Ns R + k + i Ns].  After the last stage the
// natural-order output lands in the same registers as the input pattern, so a
// forward transform can feed an inverse transform without any exchange.
//
// Pruning (zero padding of the doubled mesh, Sect. 3 of the paper): in a
// forward transform whose input is zero for indices >= P/2, the first stage's
// upper half of inputs is zero; in an inverse transform whose output is only
// needed for indices < P/2, the last stage keeps the lower half.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace nmc {

template <class R> struct CplxOf;
template <> struct CplxOf<double> { using T = double2; };
template <> struct CplxOf<float> { using T = float2; };
template <class R> using cplx = typename CplxOf<R>::T;

template <class T>
__device__ __forceinline__ T c_add(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ T c_sub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
// a * w for a twiddle w = exp(-2 pi i j / P) (DIR = -1) or its conjugate (DIR = +1)
template <int DIR, class T>
__device__ __forceinline__ T c_mul_tw(T a, T w) {
  if constexpr (DIR < 0) return T{a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
  else return T{a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// cos and sin of 2 pi j / 32 for j = 0..31 (exact decimal expansions,
// rounded once to the working precision).
struct Angle32 {
  static constexpr double c[32] = {
      1.0, 0.9807852804032304491262, 0.9238795325112867561282, 0.8314696123025452370788,
      0.7071067811865475244008, 0.5555702330196022247428, 0.3826834323650897717285, 0.1950903220161282678483,
      0.0, -0.1950903220161282678483, -0.3826834323650897717285, -0.5555702330196022247428,
      -0.7071067811865475244008, -0.8314696123025452370788, -0.9238795325112867561282, -0.9807852804032304491262,
      -1.0, -0.9807852804032304491262, -0.9238795325112867561282, -0.8314696123025452370788,
      -0.7071067811865475244008, -0.5555702330196022247428, -0.3826834323650897717285, -0.1950903220161282678483,
      0.0, 0.1950903220161282678483, 0.3826834323650897717285, 0.5555702330196022247428,
      0.7071067811865475244008, 0.8314696123025452370788, 0.9238795325112867561282, 0.9807852804032304491262};
  static constexpr double s[32] = {
      0.0, 0.1950903220161282678483, 0.3826834323650897717285, 0.5555702330196022247428,
      0.7071067811865475244008, 0.8314696123025452370788, 0.9238795325112867561282, 0.9807852804032304491262,
      1.0, 0.9807852804032304491262, 0.9238795325112867561282, 0.8314696123025452370788,
      0.7071067811865475244008, 0.5555702330196022247428, 0.3826834323650897717285, 0.1950903220161282678483,
      0.0, -0.1950903220161282678483, -0.3826834323650897717285, -0.5555702330196022247428,
      -0.7071067811865475244008, -0.8314696123025452370788, -0.9238795325112867561282, -0.9807852804032304491262,
      -1.0, -0.9807852804032304491262, -0.9238795325112867561282, -0.8314696123025452370788,
      -0.7071067811865475244008, -0.5555702330196022247428, -0.3826834323650897717285, -0.1950903220161282678483};
};

// a * exp(DIR * 2 pi i K / RR) for compile-time K/RR with RR | 32.
template <int DIR, int K, int RR, class T>
__device__ __forceinline__ T c_rot(T a) {
  using R = decltype(a.x);
  static_assert(RR >= 1 && 32 % RR == 0, "rotation by a 32nd of a turn");
  constexpr int j0 = ((K % RR) + RR) % RR * (32 / RR);
  constexpr int j = DIR < 0 ? (32 - j0) % 32 : j0;  // angle 2 pi j / 32
  if constexpr (j == 0) return a;
  else if constexpr (j == 8) return T{-a.y, a.x};   // * i
  else if constexpr (j == 16) return T{-a.x, -a.y};  // * -1
  else if constexpr (j == 24) return T{a.y, -a.x};  // * -i
  else if constexpr (j == 4) { constexpr R h = (R)Angle32::c[4]; return T{(a.x - a.y) * h, (a.x + a.y) * h}; }
  else if constexpr (j == 12) { constexpr R h = (R)Angle32::c[4]; return T{-(a.x + a.y) * h, (a.x - a.y) * h}; }
  else if constexpr (j == 20) { constexpr R h = (R)Angle32::c[4]; return T{(a.y - a.x) * h, -(a.x + a.y) * h}; }
  else if constexpr (j == 28) { constexpr R h = (R)Angle32::c[4]; return T{(a.x + a.y) * h, (a.y - a.x) * h}; }
  else {
    constexpr R c = (R)Angle32::c[j];
    constexpr R s = (R)Angle32::s[j];
    return T{a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

// In-register DFT of length RR (power of two <= 32) by radix-2 decimation in
// time; inputs with index >= NZ are taken as zero and never read, and only
// the outputs below NOUT (RR or RR/2) are formed.
// DIR = -1: forward exp(-2 pi i jk/RR); DIR = +1: inverse (unnormalised).
template <int RR, int DIR, int NZ, int NOUT = RR, class T>
__device__ __forceinline__ void dft(T* u) {
  if constexpr (RR == 1) {
    if constexpr (NZ <= 0) u[0] = T{0, 0};
  } else if constexpr (NZ <= 0) {
#pragma unroll
    for (int i = 0; i < RR; ++i) u[i] = T{0, 0};
  } else if constexpr (NZ == 1) {
#pragma unroll
    for (int i = 1; i < RR; ++i) u[i] = u[0];
  } else {
    constexpr int H = RR / 2;
    constexpr int NZE = NZ >= RR ? H : (NZ + 1) / 2;
    constexpr int NZO = NZ >= RR ? H : NZ / 2;
    T e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      if (2 * i < NZ) e[i] = u[2 * i];
      if (2 * i + 1 < NZ) o[i] = u[2 * i + 1];
    }
    dft<H, DIR, NZE>(e);
    dft<H, DIR, NZO>(o);
    if constexpr (NOUT > H) {
      [&]<int... K>(std::integer_sequence<int, K...>) {
        ((u[K] = c_add(e[K], c_rot<DIR, K, RR>(o[K])),
          u[K + H] = c_sub(e[K], c_rot<DIR, K, RR>(o[K]))), ...);
      }(std::make_integer_sequence<int, H>{});
    } else {
      [&]<int... K>(std::integer_sequence<int, K...>) {
        ((u[K] = c_add(e[K], c_rot<DIR, K, RR>(o[K]))), ...);
      }(std::make_integer_sequence<int, H>{});
    }
  }
}

// LDS view for the exchange between stages: point n of line w lives at
// re[n' * SN + w * SW] / im[...] (SoA, so every access is one scalar), with
// n' = n, or with SWZ n' = n XOR bit 3 of n (into bit 0).  SWZ is for eight
// interleaved lines (SN = 8, lanes w = lane % 8): a stage's accesses then
// touch points n of one parity per instruction, all in one half of the 32
// LDS banks, and the swizzle spreads them over both halves.
template <class R, bool SWZ = false>
struct LdsView {
  R* re;
  R* im;
  int SN, SW, w;
  __device__ __forceinline__ int at(int n) const {
    if constexpr (SWZ) n ^= (n >> 3) & 1;
    return n * SN + w * SW;
  }
  __device__ __forceinline__ void put(int n, cplx<R> v) const {
    re[at(n)] = v.x;
    im[at(n)] = v.y;
  }
  __device__ __forceinline__ cplx<R> get(int n) const {
    return cplx<R>{re[at(n)], im[at(n)]};
  }
};

// The same with the complex points interleaved (one access of 2 reals per
// point instead of one per real and imaginary part).
template <class R, bool SWZ = false>
struct LdsViewC {
  cplx<R>* a;
  int SN, SW, w;
  __device__ __forceinline__ int at(int n) const {
    if constexpr (SWZ) n ^= (n >> 3) & 1;
    return n * SN + w * SW;
  }
  __device__ __forceinline__ void put(int n, cplx<R> v) const { a[at(n)] = v; }
  __device__ __forceinline__ cplx<R> get(int n) const { return a[at(n)]; }
};

// Twiddles of a stage from powers of the first one (FP64: trades LDS reads,
// its limit, for vector products, which have room; FP32 keeps the table).
#ifndef NMC_TWIDDLE_POWERS_F64
#define NMC_TWIDDLE_POWERS_F64 1
#endif
template <class R>
constexpr bool twiddle_powers() {
  return sizeof(R) == 8 && NMC_TWIDDLE_POWERS_F64;
}

// Ordering of the LDS exchange between stages.  Workgroup barrier, or, when
// every line's threads are lanes of one wavefront (WAVE), the wait for the
// wavefront's own LDS accesses: its instructions issue in order, so once its
// writes have completed its later reads see them, and its reads are done
// before its next writes issue; waves then run without waiting for each
// other.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  else __syncthreads();
}

// One Stockham stage and, recursively, the following ones.
//  P: line length, E: points per thread, DIR: -1 forward / +1 inverse,
//  NS: product of radices already applied, FIRST: data comes from registers,
//  PIN: input index >= P/2 is zero (only valid on the first stage),
//  POUT: only outputs < P/2 are needed (last stage),
//  WAVE: a line's threads are lanes of one wavefront (lds_sync).
template <class R, int P, int E, int DIR, int NS, bool FIRST, bool PIN, bool POUT, bool WAVE, class LV, int RAD,
          int... REST>
__device__ __forceinline__ void fft_stages(cplx<R>* v, int t, const LV& lds, const cplx<R>* __restrict__ tw) {
  constexpr int TL = P / E;
  constexpr int NB = E / RAD;  // butterflies per thread in this stage
  constexpr bool LAST = sizeof...(REST) == 0;
  static_assert(E % RAD == 0, "radix must divide points per thread");
  if constexpr (!FIRST) {
    lds_sync<WAVE>();  // previous stage's writes are visible
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = lds.get(t + TL * q);
  }
  if constexpr (!LAST) lds_sync<WAVE>();  // everyone has read before anyone overwrites
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    cplx<R> u[RAD];
#pragma unroll
    for (int i = 0; i < RAD; ++i)
      if (!(FIRST && PIN) || i < RAD / 2) u[i] = v[m + i * NB];
    const int b = t + m * TL;
    const int k = b & (NS - 1);
    if constexpr (NS > 1) {
      constexpr int STEP = P / (NS * RAD);
      if constexpr (twiddle_powers<R>()) {
        // w_i = w^i from w = w_1 by products of lower powers (depth
        // log2 i + 1): one LDS read per butterfly instead of RAD - 1
        cplx<R> w[RAD];
        w[1] = tw[k * STEP];
#pragma unroll
        for (int i = 2; i < RAD; ++i) {
          const cplx<R> a = w[i / 2], b = w[i - i / 2];
          w[i] = cplx<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
        }
#pragma unroll
        for (int i = 1; i < RAD; ++i) u[i] = c_mul_tw<DIR>(u[i], w[i]);
      } else {
#pragma unroll
        for (int i = 1; i < RAD; ++i) u[i] = c_mul_tw<DIR>(u[i], tw[i * k * STEP]);
      }
    }
    dft<RAD, DIR, (FIRST && PIN) ? RAD / 2 : RAD, (LAST && POUT) ? RAD / 2 : RAD>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int i = 0; i < RAD; ++i)
        if (!POUT || i < RAD / 2) v[m + i * NB] = u[i];
    } else {
      const int base = (b / NS) * NS * RAD + k;
#pragma unroll
      for (int i = 0; i < RAD; ++i) lds.put(base + i * NS, u[i]);
    }
  }
  if constexpr (!LAST)
    fft_stages<R, P, E, DIR, NS * RAD, false, false, POUT, WAVE, LV, REST...>(v, t, lds, tw);
}

// Per-length plans: points per thread E and the radix sequence.  Narrow
// plans hold E = 8 points per thread.  Wide plans (P >= 128) hold 16:
// one LDS exchange fewer and fewer twiddle products per point, for more
// registers per thread.  Which passes take the wide plan was measured pass
// by pass (kernels.hip); NMC_WIDE_PASSES is a bit mask over PassKind.
enum PassKind {
  kPassX = 0, kPassY = 1, kPassZ = 2, kPassIY = 3, kPassIX = 4, kPassOther = 5,
  // z pass of the scaled grids (modified method), and its inverse transform
  // after the spectrum is folded by 2 or 4 (E / 2 or E / 4 points per thread)
  kPassZScaled = 6, kPassZFold2 = 7, kPassZFold4 = 8
};
#ifndef NMC_WIDE_PASSES
#define NMC_WIDE_PASSES ((1 << kPassY) | (1 << kPassZ))
#endif

template <int P> struct NarrowPlan;
template <> struct NarrowPlan<8> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8>(); } };
template <> struct NarrowPlan<16> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 2>(); } };
template <> struct NarrowPlan<32> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 4>(); } };
template <> struct NarrowPlan<64> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 8>(); } };
template <> struct NarrowPlan<128> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 4, 4>(); } };
template <> struct NarrowPlan<256> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 8, 4>(); } };
template <> struct NarrowPlan<512> { static constexpr int E = 8; template <class F> __device__ static void run(F f) { f.template go<8, 8, 8>(); } };

// Plans with 4 and 2 points per thread (the inverse after a fold).
template <int P> struct Plan4;
template <> struct Plan4<8> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 2>(); } };
template <> struct Plan4<16> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 4>(); } };
template <> struct Plan4<32> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 4, 2>(); } };
template <> struct Plan4<64> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 4, 4>(); } };
template <> struct Plan4<128> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 4, 4, 2>(); } };
template <> struct Plan4<256> { static constexpr int E = 4; template <class F> __device__ static void run(F f) { f.template go<4, 4, 4, 4>(); } };
template <int P> struct Plan2;
template <> struct Plan2<8> { static constexpr int E = 2; template <class F> __device__ static void run(F f) { f.template go<2, 2, 2>(); } };
template <> struct Plan2<16> { static constexpr int E = 2; template <class F> __device__ static void run(F f) { f.template go<2, 2, 2, 2>(); } };

template <int P> struct WidePlan;
template <> struct WidePlan<128> { static constexpr int E = 16; template <class F> __device__ static void run(F f) { f.template go<16, 8>(); } };
template <> struct WidePlan<256> { static constexpr int E = 16; template <class F> __device__ static void run(F f) { f.template go<16, 16>(); } };
template <> struct WidePlan<512> { static constexpr int E = 16; template <class F> __device__ static void run(F f) { f.template go<8, 8, 8>(); } };
// period 1024 (the scaled grids of the modified methods, their Green tables)
template <> struct WidePlan<1024> { static constexpr int E = 16; template <class F> __device__ static void run(F f) { f.template go<16, 8, 8>(); } };

#ifndef NMC_WIDE_PASSES_F64
#define NMC_WIDE_PASSES_F64 ((1 << kPassY) | (1 << kPassZ))
#endif
// FP64 wide plans only up to P = 256: they need ~200 VGPRs (two waves per
// SIMD), which the larger P = 512 tiles measured slower with.
// The scaled grids' z pass takes the wide plans from P = 128 in both
// precisions, so that the fold leaves at least 4 points per thread there.
template <class R, int P, int K>
constexpr bool wide_plan() {
  if constexpr (P >= 1024) return true;  // 16 points per thread: a line within one wavefront
  else if constexpr (K == kPassZScaled) return P >= 128;
  else if constexpr (sizeof(R) == 4) return P >= 128 && ((NMC_WIDE_PASSES >> K) & 1) != 0;
  else return P >= 128 && P <= 256 && ((NMC_WIDE_PASSES_F64 >> K) & 1) != 0;
}
template <int P, int E> struct PlanE;
template <int P> struct PlanE<P, 16> : WidePlan<P> {};
template <int P> struct PlanE<P, 8> : NarrowPlan<P> {};
template <int P> struct PlanE<P, 4> : Plan4<P> {};
template <int P> struct PlanE<P, 2> : Plan2<P> {};
template <class R, int P, int K>
struct PlanSel {
  using type = std::conditional_t<wide_plan<R, P, K>(), WidePlan<P>, NarrowPlan<P>>;
};
// after a fold by S the same threads hold E / S points of a line of P = P' / S
template <class R, int P>
struct PlanSel<R, P, kPassZFold2> {
  using type = PlanE<P, PlanSel<R, 2 * P, kPassZScaled>::type::E / 2>;
};
template <class R, int P>
struct PlanSel<R, P, kPassZFold4> {
  using type = PlanE<P, PlanSel<R, 4 * P, kPassZScaled>::type::E / 4>;
};
template <class R, int P, int K = kPassOther>
struct Plan : PlanSel<R, P, K>::type {};

template <class R, int P, int DIR, bool PIN, bool POUT, int K, bool WAVE, class LV>
struct FftRun {
  cplx<R>* v;
  int t;
  const LV* lds;
  const cplx<R>* tw;
  template <int... RS>
  __device__ __forceinline__ void go() const {
    fft_stages<R, P, Plan<R, P, K>::E, DIR, 1, true, PIN, POUT, WAVE, LV, RS...>(v, t, *lds, tw);
  }
};

// Transform one line held as v[q] = x[t + TL q] in place (natural order out),
// TL = P / Plan<R, P, K>::E.  WAVE: the line's TL threads are lanes of one
// wavefront and the caller has made the twiddle table visible to them.
template <class R, int P, int DIR, bool PIN, bool POUT, int K = kPassOther, bool WAVE = false, class LV>
__device__ __forceinline__ void fft_line(cplx<R>* v, int t, const LV& lds, const cplx<R>* __restrict__ tw) {
  Plan<R, P, K>::run(FftRun<R, P, DIR, PIN, POUT, K, WAVE, LV>{v, t, &lds, tw});
}

}  // namespace nmc
