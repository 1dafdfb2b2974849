// HIP kernels (gfx950) for the nested-mesh convolution method.
//
// Per grid (Sect. 3 of the paper) the potential is the circular convolution,
// on a doubled periodic mesh of P^3 points, of the zero-padded density with
// the periodic inverse-distance kernel.  The 3-D transform is done as five
// passes, each one launch over every grid of the solve:
//
//   X  (fwd_x): real lines along x, N nonzero of P -> P/2 complex columns;
//               the real DC and Nyquist columns are packed into column 0
//   Y  (fwd_y): lines along y, N nonzero of P -> P
//   Z  (z):     lines along z: forward, times the real Green spectrum and
//               the level scale, inverse, keep the output rows
//   I2 (inv_y): lines along y, P -> keep the output rows
//   I1 (inv_x): C2R lines along x, P/2 packed columns -> keep the output
//               cells; full grids of level >= 1 add the carried coarse
//               potential here (Sect. 4, Eq. 14)
//
// Layouts (complex, kx fastest): A[z][y][kx] (N x N x P/2), B[z][ky][kx]
// (N x P x P/2).  Strided passes give each workgroup W adjacent kx columns,
// so every global access is a run of W complex values.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft_core.hpp"
#include "kernels.h"

namespace nmc {

#ifndef NMC_Z_LDS_KB
#define NMC_Z_LDS_KB 64
#endif
#ifndef NMC_MIN_WAVES_F32
#define NMC_MIN_WAVES_F32 6
#endif
#ifndef NMC_MIN_WAVES_F32_BIG
#define NMC_MIN_WAVES_F32_BIG 1
#endif
#ifndef NMC_MIN_WAVES_F64
#define NMC_MIN_WAVES_F64 4
#endif
#ifndef NMC_MIN_WAVES_F64_WIDE
#define NMC_MIN_WAVES_F64_WIDE 1
#endif
// FP32 z pass at P = 512 through staged tiles (k_zs) and its resident waves
// per SIMD
#ifndef NMC_Z_STAGED
#define NMC_Z_STAGED 1
#endif
// FP64 z pass at P = 512 with one-row workgroups (k_z<..., ONE>)
#ifndef NMC_Z_ONE_ROW
#define NMC_Z_ONE_ROW 1
#endif
#ifndef NMC_Z_ONE_ROW_F32
#define NMC_Z_ONE_ROW_F32 0
#endif
// one-row workgroups for the scaled grids at period 1024 (both precisions)
#ifndef NMC_Z_ONE_ROW_SCALED
#define NMC_Z_ONE_ROW_SCALED 1
#endif
// FP64 passes at P = 1024 (the scaled grids) read the twiddle table from
// global memory (L2) instead of staging its 16 KB in LDS: the x, y and z
// tiles then leave room for two workgroups per CU instead of one (z pass of
// the quadrupled grids, 128^3 x 8: 8.1 -> 4.8 ms per launch on average;
// three-level solves 31 -> 45 per second)
#ifndef NMC_GLOBAL_TW_1024
#define NMC_GLOBAL_TW_1024 1
#endif
// and so do the FP64 x passes at P = 512: 32 KB of LDS per workgroup, five
// resident per CU instead of four (256^3 x 6, inverse x: full grids 0.130
// -> 0.115 ms, child-region boxes 0.109 -> 0.084 ms per launch)
#ifndef NMC_IX_GLOBAL_TW
#define NMC_IX_GLOBAL_TW 1
#endif
#ifndef NMC_X_GLOBAL_TW
#define NMC_X_GLOBAL_TW 1
#endif
template <class R, int P>
constexpr bool global_twiddles() {
  return sizeof(R) == 8 && P >= 1024 && NMC_GLOBAL_TW_1024;
}
// LDS swizzle (LdsView) of the eight interleaved lines of the one-row z
// workgroups, real and imaginary parts apart: 256^3 x 6 levels FP64, z pass
// 3.04 -> 2.99 ms.  The y passes'
// workgroups of eight FP64 columns at P = 512 have the same layout and ran
// no faster with it (1.24 ms either way), so they keep the plain one.
#ifndef NMC_Z_SWZ_ONE
#define NMC_Z_SWZ_ONE 1
#endif
// ... and with the points' real and imaginary parts interleaved (one
// 16-byte LDS access per FP64 point; 256^3 x 6: 3.06 -> 2.91 ms, where the
// swizzle no longer helps: 2.98 ms with it)
#ifndef NMC_Z_AOS
#define NMC_Z_AOS 1
#endif
#ifndef NMC_Z_AOS_SWZ
#define NMC_Z_AOS_SWZ 0
#endif
// ... in the FP64 row-pair workgroups as well (128^3 x 8: 0.381 -> 0.372
// ms, modified method 264 -> 275 solves/s); FP32 keeps the split parts
// (no change measured at 64^3 and 128^3)
#ifndef NMC_Z_AOS_ALL
#define NMC_Z_AOS_ALL 1
#endif
#ifndef NMC_Z_AOS_F32
#define NMC_Z_AOS_F32 0
#endif
#ifndef NMC_ZS_MINW_F64
#define NMC_ZS_MINW_F64 2
#endif
#ifndef NMC_ZS_MINW_F32
#define NMC_ZS_MINW_F32 4
#endif
template <class R, int P, int K>
struct Cfg {
  static constexpr int E = Plan<R, P, K>::E;
  static constexpr int TL = P / E;
  static constexpr int BYTES_PT = 2 * (int)sizeof(R);
  static constexpr int LDS = 65536;
  static constexpr int WMAX = sizeof(R) == 8 ? 16 : 32;
  static constexpr int cmin(int a, int b) { return a < b ? a : b; }
  static constexpr int WS = cmin(cmin(P / 2, WMAX), LDS / (P * BYTES_PT));  // y passes
  // z pass: two rows of W columns; W columns make one 128-byte run
  // and, up to P = 256, the workgroup stays within 512 threads so that two
  // fit a CU's registers (measured; at P = 512 the wider runs win)
  static constexpr int WZ0 = cmin(cmin(P / 2, 128 / BYTES_PT), NMC_Z_LDS_KB * 1024 / (2 * P * BYTES_PT));
  static constexpr int WZ = P >= 512 ? WZ0 : cmin(WZ0, 256 / TL > 0 ? 256 / TL : 1);
  static constexpr int WC = cmin(cmin(256 / TL, 64), LDS / (P * BYTES_PT));  // x passes
  // resident waves per SIMD the register allocation must allow (FP32: 6,
  // i.e. 80 VGPRs and three z workgroups per CU, up to P = 128; at P = 256
  // the two-stream schedule ran faster with the unconstrained allocation)
  static constexpr int MINW = sizeof(R) == 8 ? (E == 16 ? NMC_MIN_WAVES_F64_WIDE : NMC_MIN_WAVES_F64)
                                             : P <= 128 ? NMC_MIN_WAVES_F32 : NMC_MIN_WAVES_F32_BIG;
  static_assert(WS >= 1 && WZ >= 1 && WC >= 1, "tile does not fit");
};

// Copy the P twiddles exp(-2 pi i j/P) into LDS once per workgroup.  The
// first read happens in the second FFT stage, after at least one barrier.
template <class R, int P>
__device__ __forceinline__ void stage_twiddles(cplx<R>* stw, const cplx<R>* __restrict__ tw) {
  for (int j = threadIdx.x; j < P; j += blockDim.x) stw[j] = tw[j];
}

// The same for a workgroup of NTH threads, split in two: the loads are
// issued first (constructor) and the LDS writes (put) come after the
// kernel's own data loads, so that no load waits for another.  STRIDE 2
// takes the P twiddles from the table of period 2P (every second entry).
template <class R, int P, int NTH, int STRIDE = 1>
struct TwStage {
  static constexpr int K = (P + NTH - 1) / NTH;
  cplx<R> r[K];
  __device__ __forceinline__ explicit TwStage(const cplx<R>* __restrict__ tw) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = threadIdx.x + k * NTH;
      if (j < P) r[k] = tw[STRIDE * j];
    }
  }
  __device__ __forceinline__ void put(cplx<R>* stw) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = threadIdx.x + k * NTH;
      if (j < P) stw[j] = r[k];
    }
  }
};

// Restricted density of cell (cz, cy, cx) of a level's child region (cell
// c + N/4 of the level) from the restriction data F.rc: the sum over the
// finer levels k = l+1, l+2, ... of the block mean of m_k over the cell's
// footprint (Sect. 2; the unrolled cascade, kernels.h).  The footprint on
// level l+1 is the block [2c, 2c+2); on the next level it is
// [2 z - N/2, ...) twice as wide, as long as it lies inside that level.
template <class R>
__device__ __forceinline__ R restricted_at(const FieldDesc& F, int N, int cz, int cy, int cx) {
  const R* base = static_cast<const R*>(F.rc);
  const R* p = base;
  int z = 2 * cz, y = 2 * cy, x = 2 * cx;
  bool on = true;
  size_t off = 0;
  // every term's load is issued before the first is used; terms past the
  // footprint's last level read the first value and are dropped
  R t[kMaxPyramidDepth];
#pragma unroll
  for (int d = 1; d <= kMaxPyramidDepth; ++d) {
    on = on && d <= F.rdepth;
    const int nd = N >> d;
    t[d - 1] = on ? p[off + ((size_t)(z >> d) * nd + (y >> d)) * nd + (x >> d)] : base[0];
    if (!on) t[d - 1] = 0;
    z = 2 * z - N / 2;
    y = 2 * y - N / 2;
    x = 2 * x - N / 2;
    on = on && (unsigned)z < (unsigned)N && (unsigned)y < (unsigned)N && (unsigned)x < (unsigned)N;
    p += F.rslab;
    off += (size_t)nd * nd * nd;
  }
  R s = 0;
#pragma unroll
  for (int d = 0; d < kMaxPyramidDepth; ++d) s += t[d];
  return s;
}

// Input extent nin (input rows [ilo, ilo + nin) of the frame, stored
// relative to ilo by the forward passes) and output rows [olo, olo + nout)
// of a grid (FieldDesc).
struct GridGeo {
  int nin, olo, nout, ilo;
};
// DBL: a launch of scaled grids (kinds 3 and 5, scale factor S = 2 or 4:
// S N cells of the finer level's spacing spanning level l, its N input rows
// centred at (S-1) N/2, the N rows of level l left by the z pass's fold);
// kept out of the other launches' code, where the extra case measurably
// costs registers.
template <bool DBL = false>
__device__ __forceinline__ GridGeo grid_geo(int kind, int N, int S = 1) {
  if (DBL) return GridGeo{N, 0, N, (S - 1) * N / 2};
  if (kind == 0 || kind == 4) return GridGeo{N, 0, N, 0};
  if (kind == 1) return GridGeo{N / 2 + 2, 0, N / 2 + 2, 0};
  return GridGeo{N, N / 4 - 1, N / 2 + 2, 0};
}

// ---------------------------------------------------------------------------
// X pass: R2C along x with zero padding (input index >= nin is zero).
//
// Inputs of the x line (z, y) of a grid: thread t's points x = t + TL q,
// q < E/2 (the upper half is the zero padding).  Kinds 0, 3: the level's row
// with the child region restricted when rc is set (kinds 3 and 5 place it at
// x + xo of the frame); kinds 2, 4, 5: the row with the child region zeroed;
// kind 1: row of the child-region box.  An inactive line gives zeros.
template <class R, int P, bool FULLN, int K, bool DBL = false>
__device__ __forceinline__ void x_inputs(const FieldDesc& F, int N, int z, int y, bool active, int t,
                                         cplx<R>* v, int xo = 0) {
  using T = cplx<R>;
  constexpr int E = Plan<R, P, K>::E, TL = P / E;
  const R* rho = static_cast<const R*>(F.rho);
  const bool rc = F.rc != nullptr;
  const int N2 = N / 2;
  if (F.kind != 1) {
    const int lo = N / 4, hi = 3 * N / 4;
    // xo: frame offset of the row (scaled grids); kind 5 zeroes the child region
    const bool yz_in = z >= lo && z < hi && y >= lo && y < hi;
    const bool use_rc = (DBL || F.kind == 0) && rc && yz_in;
    const bool zero_c = (F.kind == 2 || F.kind == 4 || (DBL && F.kind == 5)) && yz_in;
    const size_t row = ((size_t)z * N + y) * N;
    // the level's own values first, all loads at once (a valid cell stands
    // in where the value is dropped), then the restricted child region
    R own[E / 2];
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int x = t + TL * q - xo;
      const bool xin = DBL ? (unsigned)x < (unsigned)N : x < N;
      own[q] = rho[row + ((FULLN || xin) ? x : 0)];
    }
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int x = t + TL * q - xo;
      const bool xin = DBL ? (unsigned)x < (unsigned)N : x < N;
      const bool cen = x >= lo && x < hi;
      R val = (active && (FULLN || xin) && !(zero_c && cen)) ? own[q] : (R)0;
      if (active && use_rc && cen) val = restricted_at<R>(F, N, z - lo, y - lo, x - lo);
      v[q] = T{val, 0};
    }
  } else {
    // box cell (x, y, z) is level cell (x, y, z) + N/4 - 1; the child region
    // is box cells [1, N/2 + 1) per axis
    const bool yz_in = active && z >= 1 && z <= N2 && y >= 1 && y <= N2;
    const int off = N / 4 - 1;
    const size_t row = yz_in ? ((size_t)(z + off) * N + (y + off)) * N + off + 1 : 0;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int x = t + TL * q;
      R val = 0;
      if (yz_in && x >= 1 && x <= N2) val = rc ? restricted_at<R>(F, N, z - 1, y - 1, x - 1) : rho[row + (x - 1)];
      v[q] = T{val, 0};
    }
  }
}

// Half spectrum of a transformed real x line, k = t + TL q < P/2, with the
// real DC and Nyquist values packed into k = 0.
template <class R, int P, int K>
__device__ __forceinline__ cplx<R> x_packed(const cplx<R>* v, int t, int q) {
  constexpr int E = Plan<R, P, K>::E;
  return (t == 0 && q == 0) ? cplx<R>{v[0].x, v[E / 2].x} : v[q];
}

// Value x of the lane `src` of this wavefront (a 32-bit lane permute through
// the LDS crossbar; no LDS allocation, no barrier).
__device__ __forceinline__ float lane_read(float x, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(x)));
}
__device__ __forceinline__ double lane_read(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Units (line pairs or lines) per workgroup of the x passes, and whether
// their exchanges wait per wavefront instead of per workgroup.  A line's
// threads are lanes of one wavefront, so once the workgroup has staged the
// twiddle table its wavefronts need no workgroup barrier: each takes IT
// units in turn at its own pace, and the table is staged once per IT units.
// Measured at 256^3 x 6 levels, FP64, with the twiddle table in LDS: forward
// x pass 0.755 ms with one unit per wavefront, 0.636 ms with four; the
// inverse x pass, whose carry epilogue gathers from the carried box, ran
// slower with four (0.127 -> 0.140 ms per launch).  With the FP64 table
// read from global memory (NMC_X_GLOBAL_TW, NMC_IX_GLOBAL_TW) the LDS it
// frees gives the same or better with one unit (forward 0.60 ms with one,
// two or four), so both keep one.  At P = 1024 (scaled grids, 16 points per
// lane) four units took the FP64 pass to over 300 registers and from 0.82
// to 1.0 ms.
#ifndef NMC_X_ITERS
#define NMC_X_ITERS 1
#endif
#ifndef NMC_IX_ITERS
#define NMC_IX_ITERS 1
#endif
#ifndef NMC_X_WAVE
#define NMC_X_WAVE 1
#endif
template <int P, bool INV = false>
constexpr int x_iters() { return P == 512 ? (INV ? NMC_IX_ITERS : NMC_X_ITERS) : 1; }

// PAIRS: two real lines a, b per complex transform: z = a + i b,
// Z = FFT(z), A[k] = (Z[k] + conj Z[P-k]) / 2, B[k] = (Z[k] - conj Z[P-k]) / (2i).
// The point P - k of thread t's point k = t + TL q sits in thread TL - t,
// slot E-1-q (thread 0 holds its own), read across lanes; the TL threads of a
// line are consecutive lanes of one wavefront.  Otherwise one line per
// transform (more workgroups; measured faster for FP32 below N = 128).
template <class R, int P, bool FULLN, bool PAIRS, bool DBL = false>
__global__ void __launch_bounds__((Cfg<R, P, kPassX>::WC * Cfg<R, P, kPassX>::TL))
k_fwd_x(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassX>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WC, LPW = PAIRS ? 2 : 1, IT = x_iters<P>();
  constexpr bool WAVE = NMC_X_WAVE != 0;
  static_assert(64 % TL == 0, "a line's threads must share a wavefront");
  constexpr bool GTW = global_twiddles<R, P>() || (NMC_X_GLOBAL_TW && sizeof(R) == 8 && P == 512);
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw_lds[GTW ? 1 : P];
  const cplx<R>* const stw = GTW ? tb.tw : stw_lds;
  const TwStage<R, GTW ? 1 : P, C::WC * C::TL> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = FULLN ? P / 2 : g.N, n = grid_geo<DBL>(F.kind, N, g.S).nin;
  const int nunits = n * n / LPW;  // n is even: the two lines of a pair share z
  if ((int)blockIdx.x * IT * W >= nunits) return;  // uniform: a smaller grid of a mixed launch
  const int t = threadIdx.x % TL, w = threadIdx.x / TL;
  const int xo = DBL ? (g.S - 1) * N / 2 : 0;
  const LdsView<R> lds{sre, sim, 1, P, w};
  if constexpr (!GTW) {
    tws.put(stw_lds);
    if constexpr (WAVE) __syncthreads();  // the table is complete before the first stage that reads it
  }
  // units u0 + w of the workgroup's wavefronts (a loop even of one trip
  // measurably costs registers at 16 points per lane, so IT = 1 has none)
  auto units = [&](int u0) {
    const int unit = u0 + w;
    const bool active = unit < nunits;
    const int line = active ? LPW * unit : 0;
    const int z = line / n, y = line % n;
    T va[E], v[E];
    x_inputs<R, P, FULLN, kPassX, DBL>(F, N, z, y, active, t, va, xo);
    if constexpr (PAIRS) {
      T vb[E];
      x_inputs<R, P, FULLN, kPassX, DBL>(F, N, z, y + 1, active, t, vb, xo);
#pragma unroll
      for (int q = 0; q < E / 2; ++q) v[q] = T{va[q].x, vb[q].x};
    } else {
#pragma unroll
      for (int q = 0; q < E / 2; ++q) v[q] = va[q];
    }
    fft_line<R, P, -1, true, false, kPassX, WAVE>(v, t, lds, stw);
    if constexpr (!PAIRS) {
      if (active) {
        T* A = static_cast<T*>(F.A) + ((size_t)z * n + y) * (P / 2);
#pragma unroll
        for (int q = 0; q < E / 2; ++q) A[t + TL * q] = x_packed<R, P, kPassX>(v, t, q);
      }
    } else {
      const int lane = threadIdx.x & 63;
      const int partner = (lane - t) + ((TL - t) & (TL - 1));
      T zm[E / 2];
#pragma unroll
      for (int q = 0; q < E / 2; ++q) {
        const T o = v[E - 1 - q];
        const T p = T{lane_read(o.x, partner), lane_read(o.y, partner)};
        zm[q] = t == 0 ? v[(E - q) % E] : p;
      }
      if (active) {
        T* Aa = static_cast<T*>(F.A) + ((size_t)z * n + y) * (P / 2);
        T* Ab = Aa + P / 2;
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
          const T zk = v[q], m = zm[q];
          T a = T{(R)0.5 * (zk.x + m.x), (R)0.5 * (zk.y - m.y)};
          T b = T{(R)0.5 * (zk.y + m.y), (R)0.5 * (m.x - zk.x)};
          if (t == 0 && q == 0) {  // DC and Nyquist are real: pack them
            a = T{v[0].x, v[E / 2].x};
            b = T{v[0].y, v[E / 2].y};
          }
          Aa[t + TL * q] = a;
          Ab[t + TL * q] = b;
        }
      }
    }
  };
  if constexpr (IT == 1) {
    units((int)blockIdx.x * W);
  } else {
    for (int it = 0; it < IT; ++it) {
      const int u0 = ((int)blockIdx.x * IT + it) * W;
      if (u0 >= nunits) break;  // uniform
      units(u0);
    }
  }
}

// ---------------------------------------------------------------------------
// Y pass: C2C along y, inputs y >= n zero, all P outputs kept.  DBL: a
// launch of scaled grids (kinds 3 and 5), whose input rows start at ilo.
template <class R, int P, bool FULLN, bool DBL = false>
__global__ void __launch_bounds__((Cfg<R, P, kPassY>::WS * Cfg<R, P, kPassY>::TL), (Cfg<R, P, kPassY>::MINW))
k_fwd_y(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassY>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WS, NT = (P / 2) / W;
  constexpr bool GTW = global_twiddles<R, P>();  // twiddles from global memory
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw_lds[GTW ? 1 : P];
  const cplx<R>* const stw = GTW ? tb.tw : stw_lds;
  const TwStage<R, GTW ? 1 : P, C::WS * C::TL> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const bool full = FULLN && F.kind != 1;  // nin = N = P/2: no bound checks
  const GridGeo gg = grid_geo<DBL>(F.kind, FULLN ? P / 2 : g.N, g.S);
  const int n = gg.nin;
  const int tile = blockIdx.x % NT, z = blockIdx.x / NT;
  if (z >= n) return;  // uniform: a smaller grid of a mixed launch
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int kx = tile * W + w;
  const T* A = static_cast<const T*>(F.A) + (size_t)z * n * (P / 2) + kx;
  T* B = static_cast<T*>(F.B) + (size_t)z * zrow_pitch(P, sizeof(T)) + kx;
  T v[E];
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int yy = t + TL * q - (DBL ? gg.ilo : 0);
    const bool in = full || (DBL ? (unsigned)yy < (unsigned)n : yy < n);
    const T a = A[(size_t)(in ? yy : 0) * (P / 2)];  // branch-free: a valid row, value dropped
    v[q] = in ? a : T{0, 0};
  }
  const LdsView<R> lds{sre, sim, W, 1, w};
  if constexpr (!GTW) tws.put(stw_lds);
  fft_line<R, P, -1, true, false, kPassY>(v, t, lds, stw);
#pragma unroll
  for (int q = 0; q < E; ++q) B[(size_t)(t + TL * q) * (P / 2)] = v[q];
}

// ---------------------------------------------------------------------------
// Reduction of the scaled grids (kinds 3 and 5) of the modified method
// (Sect. 7, Appendix B) to level l, taken in the spectrum.  A doubled
// (S = 2) or quadrupled (S = 4) grid has S N cells per axis of the finer
// level's spacing and spans level l: level cell j covers
// the scaled cells S j .. S j + S - 1 per axis, and its value is the mean of
// the S^3.  For a line of values x_n of period 2Q with spectrum X
// (x_n = sum_K X[K] exp(2 pi i K n / 2Q)), the pair means
// y_j = (x_2j + x_2j+1) / 2 have the period-Q spectrum
//   Y[k] = ((X[k] + X[k+Q]) + w^k (X[k] - X[k+Q])) / 2,  w = exp(2 pi i / 2Q),
// and the means of four are the pair means of the pair means.  So each
// inverse transform (z, y, x) runs at the level's period P on the spectrum
// folded log2 S times and yields level l's cells directly.
// fold_pair: Y[k] from X[k] = a, X[k+Q] = b and wc = exp(-2 pi i k / 2Q)
// (the table entry; w^k is its conjugate), times the extra factor s.
template <class R>
__device__ __forceinline__ cplx<R> fold_pair(cplx<R> a, cplx<R> b, cplx<R> wc, R s) {
  const cplx<R> d{a.x - b.x, a.y - b.y};
  const cplx<R> wd{wc.x * d.x + wc.y * d.y, wc.x * d.y - wc.y * d.x};  // conj(wc) d
  return cplx<R>{s * (a.x + b.x + wd.x), s * (a.y + b.y + wd.y)};
}

// The period-P spectrum value Y[k] of the S-means from the period-S P
// spectrum point values xs(m), m = k + P s (tw: the period-S P table).
template <class R, int P, int S, class X>
__device__ __forceinline__ cplx<R> fold_to_p(X xs, int k, const cplx<R>* __restrict__ tw) {
  if constexpr (S == 2) {
    return fold_pair<R>(xs(k), xs(k + P), tw[k], (R)0.5);
  } else {
    static_assert(S == 4, "scale 2 or 4");
    const cplx<R> lo = fold_pair<R>(xs(k), xs(k + 2 * P), tw[k], (R)0.5);
    const cplx<R> hi = fold_pair<R>(xs(k + P), xs(k + 3 * P), tw[k + P], (R)0.5);
    return fold_pair<R>(lo, hi, tw[2 * k], (R)0.5);
  }
}

// Work unit (row pair p, tile) and grid f of z-pass block b.  Consecutive
// blocks are dispatched to the 8 XCDs in turn, each with its own L2; the
// remap gives every XCD all grids of a unit back to back (the unit's spectrum
// values are then read from HBM once per XCD, not once per grid) and, where
// a tile's column run is half a 128-byte line (TP = 2), both tiles of the
// line.  Needs U (units per grid) to be a multiple of 8 TP; else identity.
__device__ __forceinline__ void z_unit(int b, int U, int nf, int TP, int& u, int& f) {
  if (U % (8 * TP) != 0) {
    u = b % U;
    f = b / U;
    return;
  }
  const int x = b % 8, s = b / 8;
  f = s % nf;
  const int j = s / nf;
  u = ((j / TP) * 8 + x) * TP + j % TP;
}

// Row r and tile of unit u of a grid of `rows` rows of NTL tiles.  With
// NMC_Z_KYFAST consecutive units step through the rows (the workgroups in
// flight then touch rows 4 KB apart, on different HBM channels, rather than
// the neighbouring tiles of one row), keeping the TP tiles that share a
// 128-byte line together; else through the tiles of a row.
#ifndef NMC_Z_KYFAST
#define NMC_Z_KYFAST 1
#endif
__device__ __forceinline__ void z_row_tile(int u, int rows, int NTL, int TP, int& r, int& tile) {
  if (NMC_Z_KYFAST && NTL % TP == 0) {
    const int v = u / TP;
    r = v % rows;
    tile = (v / rows) * TP + u % TP;
  } else {
    r = u / NTL;
    tile = u % NTL;
  }
}

// ---------------------------------------------------------------------------
// Z pass: forward along z (inputs z >= n zero), multiply by the real Green
// spectrum times the level scale, inverse along z, keep rows z < n.
// A workgroup owns the rows ky and -ky (mod P) of W adjacent kx columns.
// The packed DC/Nyquist column kx = 0 needs the value at (-ky, -kz) to
// separate the two real planes before they are multiplied by different
// spectra, an exchange through LDS with two barriers.  By default the
// workgroups of the first tile do it for their lane kx = 0.  With
// z_col0_split workgroups of their own at the start of the grid do it, each
// owning column 0 of the row pairs of W values of p, and the other
// workgroups skip it (their lane kx = 0 stores nothing).  Measured faster
// for the FP64 level grids at P = 128 and the scaled grids from P = 256;
// elsewhere the extra workgroups' latency (small launches) or their
// scattered column accesses cost as much as (FP32 level grids at P = 128)
// or more than the exchange they remove.
// SC > 1: a launch of scaled grids (kinds 3 and 5) of scale SC, whose input
// rows start at ilo; after the multiply their spectrum is folded SC times
// shorter and inverted at P / SC, which leaves the N rows of level l (the z
// means).
template <class R, int P, int SC>
constexpr bool z_col0_split() { return SC == 1 ? P == 128 && sizeof(R) == 8 : P >= 256; }
// Column-0 workgroups of a launch of nf grids, rounded up to a multiple of 8
// so that the other workgroups keep their XCD (blockIdx mod 8, see z_unit).
__host__ __device__ constexpr int z_col0_blocks(int NT, int nf) { return (NT * nf + 7) / 8 * 8; }

// ONE (FP64 level grids at P = 512, scaled grids at P = 1024): the
// workgroups other than the column-0 ones own 2 W adjacent columns of a
// single row instead of W columns of the row pair ky, -ky, so that each
// memory instruction covers runs of 2 W values (at P = 512 FP64 128-byte
// runs instead of 64-byte ones), with the same LDS tile.  The DC/Nyquist
// column is then left to the column-0 workgroups.
template <class R, int P, bool FULLN, int SC = 1, bool ONE = false>
__global__ void __launch_bounds__((2 * Cfg<R, P, SC == 1 ? kPassZ : kPassZScaled>::WZ *
                                   Cfg<R, P, SC == 1 ? kPassZ : kPassZScaled>::TL),
                                  (Cfg<R, P, SC == 1 ? kPassZ : kPassZScaled>::MINW))
k_z(FieldTable ft, PassGeom g, Tables<R> tb) {
  constexpr bool DBL = SC > 1;
  constexpr int KZ = DBL ? kPassZScaled : kPassZ;
  using C = Cfg<R, P, KZ>;
  static_assert(C::WZ == Cfg<R, P, kPassZ>::WZ, "the spectrum layout assumes the z pass's tile width");
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WZ, NT = (P / 2) / W, H = P / 2 + 1;
  __shared__ __align__(16) R sbuf[4 * W * P];
  R* const sre = sbuf;
  R* const sim = sbuf + 2 * W * P;
  constexpr bool GTW = global_twiddles<R, P>();  // twiddles from global memory
  __shared__ cplx<R> stw_lds[GTW ? 1 : P];
  const cplx<R>* const stw = GTW ? tb.tw : stw_lds;
  const TwStage<R, GTW ? 1 : P, 2 * C::WZ * C::TL> tws(tb.tw);
  constexpr int WM = ONE ? 2 * W : W, NTM = (P / 2) / WM;  // columns and tiles of a workgroup's row(s)
  constexpr int TP = WM * (int)sizeof(T) < 128 ? 2 : 1;   // tiles sharing a 128-byte line
  constexpr bool SPLIT = ONE || z_col0_split<R, P, SC>();
  const int nc0 = SPLIT ? z_col0_blocks(NT, g.nf) : 0;
  const bool col0 = SPLIT && (int)blockIdx.x < nc0;  // uniform: a column-0 workgroup
  const int t = threadIdx.x / (2 * W);
  int w = threadIdx.x % W, side = (threadIdx.x / W) & 1;
  int f, tile, p;
  if (col0) {
    if ((int)blockIdx.x >= NT * g.nf) return;  // padding
    f = blockIdx.x / NT;
    tile = 0;
    p = (blockIdx.x % NT) * W + w;
  } else if constexpr (ONE) {
    // unit (row ky, tile of WM columns); side 0 and p = ky, the row itself
    int unit;
    z_unit(blockIdx.x - nc0, NTM * P, g.nf, TP, unit, f);
    w = threadIdx.x % WM;
    side = 0;
    z_row_tile(unit, P, NTM, TP, p, tile);
  } else {
    int unit;
    z_unit(blockIdx.x - nc0, NT * (P / 2), g.nf, TP, unit, f);
    z_row_tile(unit, P / 2, NT, TP, p, tile);
  }
  const FieldDesc& F = ft.f[f];
  const bool full_in = FULLN && F.kind != 1;  // nin = N = P/2: no bound checks on loads
  const bool full = FULLN && F.kind == 0;     // nout = N = P/2 as well
  const GridGeo gg = grid_geo<DBL>(F.kind, FULLN ? P / 2 : g.N, g.S);
  const int n = gg.nin;
  const int ky = side == 0 ? p : (p == 0 ? P / 2 : P - p);  // ONE: p is any row in [0, P)
  const int kx = col0 ? 0 : tile * WM + w;
  const bool owner = !SPLIT || col0 || kx != 0;  // this lane stores its line
  const int kyp = ky <= P / 2 ? ky : P - ky;
  T* B = static_cast<T*>(F.B) + (size_t)ky * (P / 2) + kx;  // row z at + z ZS
  constexpr size_t ZS = zrow_pitch(P, sizeof(T));
  // rows z >= n are zero (no load)
  T v[E];
  if (full_in) {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) v[q] = B[(size_t)(t + TL * q) * ZS];
  } else {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int zz = t + TL * q - (DBL ? gg.ilo : 0);
      v[q] = (DBL ? (unsigned)zz < (unsigned)n : zz < n) ? B[(size_t)zz * ZS] : T{0, 0};
    }
  }
  // spectrum values of this thread's points (the spectrum is even in kz:
  // kz = t + TL q reads row kz for q < E/2 and row P - kz = P/2 - t - TL (q - E/2)
  // above)
  const R* gcol = tb.gz + (size_t)(kyp * NT + kx / W) * H * W + kx % W;
  const R* glo = gcol + t * W;
  const R* ghi = gcol + (P / 2 - t) * W;
  // FP32: fetched after the forward transform, so that they hold no
  // registers during it (the earlier fetch cost a resident workgroup);
  // FP64: fetched with the data (measured faster)
  constexpr bool late = sizeof(R) == 4;
  R ga[E];
  auto fetch_spectrum = [&]() {
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      ga[q] = glo[TL * q * W];
      ga[q + E / 2] = ghi[-TL * q * W];
    }
  };
  if constexpr (!late) fetch_spectrum();
  // ONE: line w < 2 W, side 0
  constexpr bool SWZV = ONE && NMC_Z_SWZ_ONE && 2 * W == 8;
  const auto lds = [&] {
    if constexpr (NMC_Z_AOS && (ONE || NMC_Z_AOS_ALL) && (sizeof(R) == 8 || NMC_Z_AOS_F32))
      return LdsViewC<R, SWZV && NMC_Z_AOS_SWZ>{reinterpret_cast<cplx<R>*>(sbuf), 2 * W, 1, w + W * side};
    else
      return LdsView<R, SWZV>{sre, sim, 2 * W, 1, w + W * side};
  }();
  if constexpr (!GTW) tws.put(stw_lds);
  fft_line<R, P, -1, true, false, KZ>(v, t, lds, stw);
  if constexpr (late) fetch_spectrum();

  const R sc = (R)F.scale;
  // the exchange: every lane of a column-0 workgroup, else lane kx = 0 of the
  // first tile; point kz of line (side, w) goes to LDS at (side P + kz) XW + w
  constexpr int XW = SPLIT ? W : 1;
  bool plain = true;
  if (SPLIT ? col0 : tile == 0) {  // uniform per workgroup
    __syncthreads();  // the forward transform's last LDS reads are done
    if (SPLIT || w == 0) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int kz = t + TL * q;
        sre[(side * P + kz) * XW + w] = v[q].x;
        sim[(side * P + kz) * XW + w] = v[q].y;
      }
    }
    __syncthreads();
    plain = !SPLIT && w != 0;
  }
  if (plain) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const R gv = sc * ga[q];
      v[q] = T{v[q].x * gv, v[q].y * gv};
    }
  } else {
    // column 0 holds U + iV (U, V: spectra of the real DC and Nyquist planes);
    // with Cm = conj(value at -k): U = (C + Cm)/2, V = (C - Cm)/(2i), and the
    // product is g0 U + i gN V = (g0+gN)/2 C + (g0-gN)/2 Cm.
    const int ps = p == 0 ? side : 1 - side;  // row holding -ky
    const R* gn = tb.gn + (size_t)kyp * H;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int kz = t + TL * q;
      const int nkz = (P - kz) & (P - 1);
      const T cm = T{sre[(ps * P + nkz) * XW + w], -sim[(ps * P + nkz) * XW + w]};
      const R g0 = ga[q], gnv = gn[kz <= P / 2 ? kz : P - kz];
      const R a = sc * (R)0.5 * (g0 + gnv), b = sc * (R)0.5 * (g0 - gnv);
      v[q] = T{a * v[q].x + b * cm.x, a * v[q].y + b * cm.y};
    }
  }
  if constexpr (!DBL) {
    fft_line<R, P, +1, false, true, kPassZ>(v, t, lds, stw);
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int zz = t + TL * q;
      if (owner && (full || (zz >= gg.olo && zz < gg.olo + gg.nout))) B[zz * ZS] = v[q];
    }
  } else {
    // fold: point kz + (P/SC) s of this thread is its slot q + s E/SC
    constexpr int EF = E / SC, PF = P / SC, KF = SC == 2 ? kPassZFold2 : kPassZFold4;
    static_assert(Plan<R, PF, KF>::E == EF, "fold plan");
    __shared__ cplx<R> stw2[PF];  // exp(-2 pi i j / PF): every SC-th twiddle
    for (int j = threadIdx.x; j < PF; j += blockDim.x) stw2[j] = stw[SC * j];
    T u[EF];
#pragma unroll
    for (int q = 0; q < EF; ++q) {  // fold_to_p with the points in registers
      const int kz = t + TL * q;
      if constexpr (SC == 2) {
        u[q] = fold_pair<R>(v[q], v[q + EF], stw[kz], (R)0.5);
      } else {
        const T lo = fold_pair<R>(v[q], v[q + 2 * EF], stw[kz], (R)0.5);
        const T hi = fold_pair<R>(v[q + EF], v[q + 3 * EF], stw[kz + PF], (R)0.5);
        u[q] = fold_pair<R>(lo, hi, stw[2 * kz], (R)0.5);
      }
    }
    // the first stage's LDS writes follow a barrier, after the stw2 writes
    fft_line<R, PF, +1, false, true, KF>(u, t, lds, stw2);
    const int Nl = g.N;
#pragma unroll
    for (int q = 0; q < EF / 2; ++q) {
      const int zz = t + TL * q;
      if (owner && zz < Nl) B[(size_t)zz * ZS] = u[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Z pass at P = 512 through staged tiles (level grids; used for FP32, where
// it ran the 256^3 x 6 launch in 1.72 ms against k_z's 1.81 ms, both at the
// unpadded row pitch; for FP64 its 220 registers leave two wavefronts per
// SIMD and k_z stays faster, 3.47 against 3.73 ms).
//
// A grid's z rows are about 2 MB apart (one z row of B holds P (P/2) values,
// zrow_pitch), and what HBM delivers for such rows depends on the contiguous
// run each memory instruction covers: at the power-of-two pitch a plain read
// and write of B on the GPU moves 2.7 TB/s with 64-byte runs (k_z's: 4 FP64
// or 8 FP32 adjacent columns per lane group), 4.0 TB/s with 128-byte runs
// and 5.0 TB/s with 256-byte runs.  Here a
// workgroup first stages the tile [row ky, -ky][z][CS columns] through LDS
// with 128-byte runs, then each wavefront transforms four whole lines with
// 32 points per lane: radix 16 then radix 32, one exchange per transform,
// through LDS rows of its own in the same space (no workgroup barrier between
// the staging steps).  The results leave through the tile the same way.
// Wavefront j owns columns 4 (j % (NW/2)) + w of the tile in row ky = p
// (j < NW/2) or -p (-0 is row P/2); lane (w, t) = (lane % 4, lane / 4)
// holds the points kz = t + 16 q, q = 0..31.  Tile 0 (with column kx = 0,
// which packs the real DC and Nyquist planes) is left to a launch of its own
// (COL0), where the two rows' column-0 lines meet after the forward
// transform.
namespace zs {
constexpr int P = 512, E = 32, TL = 16, LW = 4;
constexpr int ROWS = P + P / 16;  // exchange rows of a wavefront: a padding row after every 16 points
template <class R>
struct Geo {
  static constexpr int CS = 128 / (2 * (int)sizeof(R));  // columns per row: one 128-byte run
  static constexpr int NW = 2 * CS / LW;                  // wavefronts (both rows, four lines each)
  static constexpr int NT = 64 * NW;
  static constexpr int TILES = (P / 2) / CS;
  static constexpr int UNITS = (P / 2) * TILES;           // (row pair p, tile) per grid
  static constexpr int XM = CS / LW - 1;                   // column swizzle of the tile by z
  static constexpr int ZR = NT / (2 * CS);                // z rows per staging round
  static constexpr int TILE_BYTES = 2 * (P / 2) * CS * 2 * (int)sizeof(R);
  static constexpr int EX_BYTES = NW * ROWS * LW * (int)sizeof(R);
  static constexpr int LDS = TILE_BYTES > EX_BYTES ? TILE_BYTES : EX_BYTES;
  static_assert(ZR == 16, "staging rounds of 16 z rows");
};
}  // namespace zs

// Makes this wavefront's LDS writes visible to all its lanes and keeps the
// compiler from moving LDS accesses across it (every lane reaches it).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// w^i, i = 0..31, for w = exp(-2 pi i t / 512) (the table entry t; DIR = +1
// uses the conjugates): w^(8a + b) = w^(8a) w^b, with w^b (b < 8) products
// of at most three table values and w^(8a) from the table.  Applied to u[i]
// in place.  The lane index is made opaque first, so that each transform
// forms its own (cheap) instead of holding the forward's across the multiply.
template <int DIR, class R>
__device__ __forceinline__ void zs_twiddle(cplx<R>* u, int t, const cplx<R>* __restrict__ tw) {
  using T = cplx<R>;
  auto mul = [](T a, T b) { return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; };
  asm volatile("" : "+v"(t));
  T p[8];
  p[1] = tw[t];
  p[2] = mul(p[1], p[1]);
  p[3] = mul(p[1], p[2]);
  p[4] = mul(p[2], p[2]);
  p[5] = mul(p[1], p[4]);
  p[6] = mul(p[2], p[4]);
  p[7] = mul(p[3], p[4]);
#pragma unroll
  for (int b = 1; b < 8; ++b) u[b] = c_mul_tw<DIR>(u[b], p[b]);
#pragma unroll
  for (int a = 1; a < 4; ++a) {
    const T wa = tw[(8 * a * t) & (zs::P - 1)];
    u[8 * a] = c_mul_tw<DIR>(u[8 * a], wa);
#pragma unroll
    for (int b = 1; b < 8; ++b) u[8 * a + b] = c_mul_tw<DIR>(u[8 * a + b], mul(wa, p[b]));
  }
}

// The exchange between the two stages: slot s = 16 m + i of this lane holds
// point n = 16 (t + 16 m) + i of its line; afterwards slot q holds point
// t + 16 q.  Point n lives in row n + n / 16 of `ex` (this wavefront's
// ROWS x LW values); one component at a time, every address a lane base
// plus a constant.
template <class R>
__device__ __forceinline__ void zs_exchange(cplx<R>* v, R* ex, int w, int t) {
  using namespace zs;
  R tmp[E];
  R* const wb = ex + (17 * t) * LW + w;  // row of n = 16 t + 256 m + i: 17 t + 272 m + i
  R* const rb = ex + (t + (t >> 4)) * LW + w;  // row of t + 16 q: t + 17 q (t < 16)
#pragma unroll
  for (int s = 0; s < E; ++s) wb[(272 * (s / 16) + s % 16) * LW] = v[s].x;
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < E; ++q) tmp[q] = rb[17 * q * LW];
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < E; ++s) wb[(272 * (s / 16) + s % 16) * LW] = v[s].y;
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = cplx<R>{tmp[q], rb[17 * q * LW]};
  wave_lds_sync();
}

// One transform of a line held as v[q] = x[t + 16 q] (natural order out, in
// the same slots).  Forward: inputs q >= 16 are zero (PIN).  Inverse: only
// the outputs q < 16 are formed (POUT).  Stockham stages: radix 16 over the
// butterflies b = t + 16 m (inputs x[b + 32 i] = slot m + 2 i, outputs
// y[16 b + i]), then radix 32 over b = t (inputs y[t + 16 i], twiddles w^i
// with w = exp(-+2 pi i t / 512), outputs x[t + 16 i]).
template <int DIR, class R>
__device__ __forceinline__ void zs_fft(cplx<R>* v, R* ex, int w, int t, const cplx<R>* __restrict__ tw) {
  using T = cplx<R>;
  constexpr bool PIN = DIR < 0, POUT = DIR > 0;
  T y[zs::E];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    T u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (!PIN || i < 8) u[i] = v[m + 2 * i];
    dft<16, DIR, PIN ? 8 : 16>(u);
#pragma unroll
    for (int i = 0; i < 16; ++i) y[16 * m + i] = u[i];
  }
  zs_exchange<R>(y, ex, w, t);
  zs_twiddle<DIR, R>(y, t, tw);
  dft<32, DIR, 32, POUT ? 16 : 32>(y);
#pragma unroll
  for (int q = 0; q < (POUT ? 16 : 32); ++q) v[q] = y[q];
}

template <class R, bool FULLN, bool COL0>
__device__ __forceinline__ void zs_tile(const FieldTable& ft, const PassGeom& g, const Tables<R>& tb, int f, int p,
                                        int tl, char* lds) {
  using namespace zs;
  using G = Geo<R>;
  using T = cplx<R>;
  constexpr int CS = G::CS, NW = G::NW, XM = G::XM, ZR = G::ZR;
  constexpr int H = P / 2 + 1, W = Cfg<R, P, kPassZ>::WZ, NTL = (P / 2) / W;  // spectrum layout tiles
  T* const tile = reinterpret_cast<T*>(lds);  // [side][z][column ^ swizzle]
  const int lane = threadIdx.x % 64, j = threadIdx.x / 64;
  const int w = lane % LW, t = lane / LW;
  const FieldDesc& F = ft.f[f];
  const bool full_in = FULLN && F.kind != 1;
  const bool full = FULLN && F.kind == 0;
  const GridGeo gg = grid_geo<false>(F.kind, FULLN ? P / 2 : g.N);
  const int n = gg.nin;
  auto row_of = [&](int side) { return side == 0 ? p : (p == 0 ? P / 2 : P - p); };
  constexpr unsigned ZS = (unsigned)(zrow_pitch(P, sizeof(T)) * sizeof(T));  // bytes between z rows of B
  char* const B = static_cast<char*>(F.B);
  // staging lanes: column c, z rows zr + 16 k, row `sside` of the pair
  const int c = threadIdx.x % CS, zr = (threadIdx.x / CS) % ZR, sside = threadIdx.x / (CS * ZR);
  const unsigned gb = (unsigned)((row_of(sside) * (P / 2) + tl * CS + c) * sizeof(T)) + (unsigned)zr * ZS;
  T* const st = tile + (sside * (P / 2) + zr) * CS + (c ^ ((zr & XM) << 2));
#pragma unroll
  for (int k = 0; k < (P / 2) / ZR; ++k) {
    const int z = zr + ZR * k;
    T val = T{0, 0};
    if (full_in || z < n) val = *reinterpret_cast<const T*>(B + gb + (unsigned)k * ZR * ZS);
    st[k * ZR * CS] = val;
  }
  __syncthreads();
  // this wavefront's four lines: row `side`, tile columns 4 q4 + w
  const int side = j / (NW / 2), q4 = j % (NW / 2);
  const int col = 4 * q4 + w, kx = tl * CS + col;
  const int ky = row_of(side), kyp = ky <= P / 2 ? ky : P - ky;
  T v[E];
  {
    const T* const rt = tile + (side * (P / 2) + t) * CS + (col ^ ((t & XM) << 2));
#pragma unroll
    for (int q = 0; q < E / 2; ++q) v[q] = rt[q * TL * CS];
#pragma unroll
    for (int q = E / 2; q < E; ++q) v[q] = T{0, 0};
  }
  __syncthreads();  // the tile's space is the wavefronts' exchange rows from here
  R* const ex = reinterpret_cast<R*>(lds) + j * ROWS * LW;
  // spectrum of this lane's points: row kz = t + 16 q for q < 16, and
  // P - kz = (P - t) - 16 q from q = 16 on
  const char* const gz = reinterpret_cast<const char*>(tb.gz);
  const unsigned goff = (unsigned)(((kyp * NTL + kx / W) * H * W + kx % W) * sizeof(R));
  const unsigned glo = goff + (unsigned)(t * W * sizeof(R)), ghi = goff + (unsigned)((P - t) * W * sizeof(R));
  auto spectrum = [&](int q) {
    constexpr unsigned RS = TL * W * sizeof(R);  // bytes per 16 spectrum rows
    return *reinterpret_cast<const R*>(gz + (q < E / 2 ? glo + q * RS : ghi - q * RS));
  };
  zs_fft<-1, R>(v, ex, w, t, tb.tw);
  const R sc = (R)F.scale;
  if constexpr (!COL0) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const R gv = sc * spectrum(q);
      v[q] = T{v[q].x * gv, v[q].y * gv};
    }
  } else {
    // kx = 0 holds U + iV (U, V: spectra of the real DC and Nyquist planes);
    // with Cm = conj(value at (-ky, -kz)): U = (C + Cm)/2, V = (C - Cm)/(2i),
    // and the product g0 U + i gN V is (g0 + gN)/2 C + (g0 - gN)/2 Cm.  The
    // rows' column-0 lines (lane w = 0 of wavefronts 0 and NW/2) meet in
    // wavefront 0's exchange rows; row -ky is the other one, or the same
    // for p = 0 (rows 0 and P/2 are their own negatives).
    R* const c0 = reinterpret_cast<R*>(lds);  // [side][component][kz]
    __syncthreads();  // every forward transform is done with its rows
    if (kx == 0) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        c0[(2 * side) * P + t + TL * q] = v[q].x;
        c0[(2 * side + 1) * P + t + TL * q] = v[q].y;
      }
    }
    __syncthreads();
    if (kx == 0) {
      const int ps = p == 0 ? side : 1 - side;
      const R* gn = tb.gn + (size_t)kyp * H;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int kz = t + TL * q, nkz = (P - kz) & (P - 1);
        const T cm = T{c0[(2 * ps) * P + nkz], -c0[(2 * ps + 1) * P + nkz]};
        const R g0 = spectrum(q), gnv = gn[kz <= P / 2 ? kz : P - kz];
        const R a = sc * (R)0.5 * (g0 + gnv), b = sc * (R)0.5 * (g0 - gnv);
        v[q] = T{a * v[q].x + b * cm.x, a * v[q].y + b * cm.y};
      }
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const R gv = sc * spectrum(q);
        v[q] = T{v[q].x * gv, v[q].y * gv};
      }
    }
    __syncthreads();  // wavefront 0's rows are its exchange rows again
  }
  zs_fft<+1, R>(v, ex, w, t, tb.tw);
  __syncthreads();  // every inverse transform is done with its rows
  {
    T* const wt = tile + (side * (P / 2) + t) * CS + (col ^ ((t & XM) << 2));
#pragma unroll
    for (int q = 0; q < E / 2; ++q) wt[q * TL * CS] = v[q];
  }
  __syncthreads();
  unsigned sb = gb;
  asm volatile("" : "+v"(sb));  // not kept across the transforms
#pragma unroll
  for (int k = 0; k < (P / 2) / ZR; ++k) {
    const int z = zr + ZR * k;
    if (full || (z >= gg.olo && z < gg.olo + gg.nout))
      *reinterpret_cast<T*>(B + sb + (unsigned)k * ZR * ZS) = st[k * ZR * CS];
  }
}

// One launch: the first P/2 nf workgroups take the tiles 0 (with column
// kx = 0), the others the tiles 1.. of their unit (tile 0's exit at once).
// The two paths are separate instances, so the column-0 exchange costs the
// other tiles no registers.
template <class R, bool FULLN>
__global__ void __launch_bounds__(zs::Geo<R>::NT, (sizeof(R) == 8 ? NMC_ZS_MINW_F64 : NMC_ZS_MINW_F32))
k_zs(FieldTable ft, PassGeom g, Tables<R> tb) {
  using G = zs::Geo<R>;
  __shared__ __align__(16) char lds[G::LDS];
  const int c0_blocks = (zs::P / 2) * g.nf;  // a multiple of 8: the others keep their XCD (z_unit)
  if ((int)blockIdx.x >= c0_blocks) {
    int unit, f;
    z_unit(blockIdx.x - c0_blocks, G::UNITS, g.nf, 1, unit, f);
    int p, tl;
    z_row_tile(unit, zs::P / 2, G::TILES, 1, p, tl);
    if (tl == 0) return;  // whole workgroup
    zs_tile<R, FULLN, false>(ft, g, tb, f, p, tl, lds);
  } else {
    zs_tile<R, FULLN, true>(ft, g, tb, blockIdx.x / (zs::P / 2), blockIdx.x % (zs::P / 2), 0, lds);
  }
}

// ---------------------------------------------------------------------------
// I2 pass: inverse along y over rows z < n; keep rows y < n.
template <class R, int P, bool FULLN>
__global__ void __launch_bounds__((Cfg<R, P, kPassIY>::WS * Cfg<R, P, kPassIY>::TL), (Cfg<R, P, kPassIY>::MINW))
k_inv_y(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassIY>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WS, NT = (P / 2) / W;
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw[P];
  const TwStage<R, P, C::WS * C::TL> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const bool full = FULLN && F.kind == 0;  // nout = N = P/2: no bound checks
  const GridGeo gg = grid_geo(F.kind, FULLN ? P / 2 : g.N);
  const int r = blockIdx.x / NT;
  if (r >= gg.nout) return;  // uniform: a smaller grid of a mixed launch
  const int z = gg.olo + r;
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int kx = (blockIdx.x % NT) * W + w;
  const T* B = static_cast<const T*>(F.B) + (size_t)z * zrow_pitch(P, sizeof(T)) + kx;
  T* A = static_cast<T*>(F.A) + (size_t)z * gg.nin * (P / 2) + kx;
  T v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) v[q] = B[(size_t)(t + TL * q) * (P / 2)];
  const LdsView<R> lds{sre, sim, W, 1, w};
  tws.put(stw);
  fft_line<R, P, +1, false, true, kPassIY>(v, t, lds, stw);
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int yy = t + TL * q;
    if (full || (yy >= gg.olo && yy < gg.olo + gg.nout)) A[(size_t)yy * (P / 2)] = v[q];
  }
}

// ---------------------------------------------------------------------------
// I1 pass: C2R along x.  Child-region grids (kind 1) write their potential C
// on the stencil box.  Full grids write Phi(Omega^l) = Phi^l + Prolong(S_{l-1})
// (Sect. 4, Eq. 14) and, on the stencil box of a level that has a finer one,
// the next carry S_l = Phi(Omega^l) - C_l.  The carry is Eqs. 3-6 applied to
// every fine cell: parent c = N/4 + f/2, neighbour c + s with s = +1 for odd
// f and -1 for even f per axis, 3/4 and 1/4 weights along the diagonal.
template <class R>
__device__ __forceinline__ void two_sum(R a, R b, R& s, R& e) {
  s = a + b;
  const R bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Points x = t + TL q of the Hermitian extension of a packed half spectrum
// (row[k], k < P/2, with the real DC and Nyquist values in row[0]); every
// load is issued without a branch, an inactive line reads row 0 and drops it.
template <class R, int P, int K, class Row>
__device__ __forceinline__ void hermitian_inputs(Row row, bool active, int t, cplx<R>* v) {
  using T = cplx<R>;
  constexpr int E = Plan<R, P, K>::E, TL = P / E;
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int k = t + TL * q;  // < P/2; k = 0 holds the real DC value in .x
    const T m = row(k);
    v[q] = !active ? T{0, 0} : (k == 0 ? T{m.x, 0} : m);
  }
#pragma unroll
  for (int q = E / 2; q < E; ++q) {
    const int kk = P - (t + TL * q);  // in (0, P/2]; P/2 is the Nyquist value in row[0].y
    const T m = row(kk == P / 2 ? 0 : kk);
    v[q] = !active ? T{0, 0} : (kk == P / 2 ? T{m.y, 0} : T{m.x, -m.y});
  }
}

// Rows of the carried box S (NS cells per axis) for level cell (z, y): ii
// at the parent's z and y, jj at the neighbours' (c + s per axis, Eqs. 3-6);
// the mixed rows (parent z, neighbour y) and (neighbour z, parent y) are
// ii + dyn and jj - dyn.
struct CarryRows {
  size_t ii, jj;
  int dyn;
};
__device__ __forceinline__ CarryRows carry_rows(int z, int y, int NS) {
  const int iz = z / 2 + 1, iy = y / 2 + 1;
  const int jz = iz + ((z & 1) ? 1 : -1), jy = iy + ((y & 1) ? 1 : -1);
  return CarryRows{((size_t)iz * NS + iy) * NS, ((size_t)jz * NS + jy) * NS, (jy - iy) * NS};
}

// Prolong(S_{l-1}) at level cell x of the rows cr of the carried box S, as
// s + l.  Default, Eqs. 3-6 applied to every fine cell: 3/4 of the parent
// plus 1/4 of the diagonal neighbour.  tri (NMC_PROLONG_TRILINEAR): the
// tensor-product rule, weights 3/4 (parent) and 1/4 (neighbour) per axis
// over the 8 surrounding cells.  FP64 and the uncompensated FP32 path give
// the plain weighted sum and l = 0; the compensated path forms each product
// exactly (FMA), adds them with TwoSum and keeps the rounding errors plus the
// carried lo terms in l.
template <class R, bool TRI>
__device__ __forceinline__ void carried(bool comp, const R* S, const R* Sl, const CarryRows& cr, int x, R& s,
                                        R& l) {
  const int ix = x / 2 + 1, jx = ix + ((x & 1) ? 1 : -1);
  if constexpr (!TRI) {
    const R a = S[cr.ii + ix], b = S[cr.jj + jx];
    if (sizeof(R) == 8 || !comp) {
      s = (R)0.75 * a + (R)0.25 * b;
      l = 0;
    } else {
      const R p1 = (R)0.75 * a;
      const R e1 = fma((R)0.75, a, -p1);
      R e2;
      two_sum(p1, (R)0.25 * b, s, e2);
      l = e1 + e2;
      if (Sl) l += (R)0.75 * Sl[cr.ii + ix] + (R)0.25 * Sl[cr.jj + jx];
    }
  } else {
    const size_t ij = cr.ii + cr.dyn, ji = cr.jj - cr.dyn;
    const size_t at[8] = {cr.ii + ix, cr.ii + jx, ij + ix, ij + jx, ji + ix, ji + jx, cr.jj + ix, cr.jj + jx};
    const R w[8] = {(R)27 / 64, (R)9 / 64, (R)9 / 64, (R)3 / 64, (R)9 / 64, (R)3 / 64, (R)3 / 64, (R)1 / 64};
    R a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = S[at[i]];
    s = 0;
    l = 0;
    if (sizeof(R) == 8 || !comp) {
#pragma unroll
      for (int i = 0; i < 8; ++i) s += w[i] * a[i];
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const R p = w[i] * a[i];
        const R e = fma(w[i], a[i], -p);
        R t, e2;
        two_sum(s, p, t, e2);
        s = t;
        l += e + e2;
      }
      if (Sl) {
#pragma unroll
        for (int i = 0; i < 8; ++i) l += w[i] * Sl[at[i]];
      }
    }
  }
}

// Outputs of the inverse-transformed x line (z, y) of a grid (zr, yr: its
// row within the output box).  Kinds 1 and 2 write the box; kinds 0 and 4
// write Phi(Omega^l) = Phi^l + Prolong(S_{l-1}) (kind 4: the hole potential,
// no carry) and, on the stencil box of a level with a finer one, S_l =
// Phi(Omega^l) - C_l (child-region boxes) or the hole potential itself
// (kind 4, C null).
template <class R, int P, int K, bool TRI>
__device__ __forceinline__ void ix_outputs(const FieldDesc& F, int N, const GridGeo& gg, int z, int y,
                                           int zr, int yr, int t, const cplx<R>* v) {
  constexpr int E = Plan<R, P, K>::E, TL = P / E;
  const int n = gg.nout;
  R* out = static_cast<R*>(F.out);
  if (F.kind == 1 || F.kind == 2) {  // box output (C or the hole potential)
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int x = t + TL * q;
      if (x >= gg.olo && x < gg.olo + n) out[((size_t)zr * n + yr) * n + (x - gg.olo)] = v[q].x;
    }
    return;
  }
  const int NS = N / 2 + 2, blo = N / 4 - 1;
  const R* S = static_cast<const R*>(F.S);
  const R* Sl = static_cast<const R*>(F.Slo);
  R* So = static_cast<R*>(F.Sout);
  R* Slo = static_cast<R*>(F.Slo_out);
  const R* Cb = static_cast<const R*>(F.C);
  const bool yz_box = So && z >= blo && z < blo + NS && y >= blo && y < blo + NS;
  const CarryRows cr = carry_rows(z, y, NS);  // carry source rows for this (y, z)
  const size_t brow = ((size_t)(z - blo) * NS + (y - blo)) * NS - blo;
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int x = t + TL * q;
    if (x >= N) continue;
    const R val = v[q].x;
    R hi = val, lo = 0;  // Phi(Omega^l) as an unevaluated sum hi + lo
    if (S) {
      R s1, l;
      carried<R, TRI>(F.comp, S, Sl, cr, x, s1, l);
      if (sizeof(R) == 8 || !F.comp) {
        hi = val + s1;
      } else {
        R s2, e3;
        two_sum(val, s1, s2, e3);
        hi = s2;
        lo = e3 + l;
      }
    }
    out[((size_t)z * N + y) * N + x] = hi + lo;
    if (yz_box && x >= blo && x < blo + NS) {
      const size_t bi = brow + x;
      const R cb = Cb ? Cb[bi] : (R)0;
      if (sizeof(R) == 8 || !F.comp) {
        So[bi] = hi - cb;
        if (Slo) Slo[bi] = 0;
      } else {
        R d, e;
        two_sum(hi, -cb, d, e);
        e += lo;
        const R dh = d + e;
        So[bi] = dh;
        if (Slo) Slo[bi] = e - (dh - d);
      }
    }
  }
}

// PAIRS: two output lines a, b per complex transform: with A, B their half
// spectra (Hermitian), Z[k] = A[k] + i B[k] for all k and IFFT(Z) = a + i b.
// Otherwise one line per transform (its imaginary part unused), which keeps
// twice the workgroups and half the epilogue per thread (measured faster for
// the full grids' carry epilogue below N = 256).
template <class R, int P, bool PAIRS, bool TRI>
__global__ void __launch_bounds__((Cfg<R, P, kPassIX>::WC * Cfg<R, P, kPassIX>::TL))
k_inv_x(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassIX>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WC, LPW = PAIRS ? 2 : 1;  // lines per transform
  constexpr int IT = x_iters<P, true>();
  constexpr bool WAVE = NMC_X_WAVE != 0;
  static_assert(64 % TL == 0, "a line's threads must share a wavefront");
  constexpr bool GTW = global_twiddles<R, P>() || (NMC_IX_GLOBAL_TW && sizeof(R) == 8 && P == 512);
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw_lds[GTW ? 1 : P];
  const cplx<R>* const stw = GTW ? tb.tw : stw_lds;
  const TwStage<R, GTW ? 1 : P, C::WC * C::TL> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = g.N;
  const GridGeo gg = grid_geo(F.kind, N);
  const int n = gg.nout;
  const int nunits = n * n / LPW;  // n is even: the two lines of a pair share z
  if ((int)blockIdx.x * IT * W >= nunits) return;  // uniform: a smaller grid of a mixed launch
  const int t = threadIdx.x % TL, w = threadIdx.x / TL;
  const LdsView<R> lds{sre, sim, 1, P, w};
  if constexpr (!GTW) {
    tws.put(stw_lds);
    if constexpr (WAVE) __syncthreads();  // the table is complete before the first stage that reads it
  }
  auto units = [&](int u0) {  // as in k_fwd_x
    const int unit = u0 + w;
    const bool active = unit < nunits;
    const int line = active ? LPW * unit : 0;
    const int zr = line / n, yr = line % n;  // within the output box
    const int z = gg.olo + zr, y = gg.olo + yr;
    const T* ra = static_cast<const T*>(F.A) + ((size_t)z * gg.nin + y) * (P / 2);
    const T* rb = ra + P / 2;
    // packed half spectra: k = 0 holds the real DC (.x) and Nyquist (.y)
    // values; every load is issued without a branch (inactive units read
    // row 0 and drop it)
    T v[E];
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int k = t + TL * q;
      T a = ra[k], b = PAIRS ? rb[k] : T{0, 0};
      if (k == 0) {
        a.y = 0;
        b.y = 0;
      }
      v[q] = active ? T{a.x - b.y, a.y + b.x} : T{0, 0};
    }
#pragma unroll
    for (int q = E / 2; q < E; ++q) {
      const int kk = P - (t + TL * q);  // in (0, P/2]
      const int idx = kk == P / 2 ? 0 : kk;
      T a = ra[idx], b = PAIRS ? rb[idx] : T{0, 0};
      if (kk == P / 2) {
        a = T{a.y, 0};
        b = T{b.y, 0};
      }
      v[q] = active ? T{a.x + b.y, b.x - a.y} : T{0, 0};  // conj(A) + i conj(B)
    }
    fft_line<R, P, +1, false, true, kPassIX, WAVE>(v, t, lds, stw);
    if (active) {
      ix_outputs<R, P, kPassIX, TRI>(F, N, gg, z, y, zr, yr, t, v);
      if constexpr (PAIRS) {
        T vb[E / 2];
#pragma unroll
        for (int q = 0; q < E / 2; ++q) vb[q] = T{v[q].y, 0};
        ix_outputs<R, P, kPassIX, TRI>(F, N, gg, z, y + 1, zr, yr + 1, t, vb);
      }
    }
  };
  if constexpr (IT == 1) {
    units((int)blockIdx.x * W);
  } else {
    for (int it = 0; it < IT; ++it) {
      const int u0 = ((int)blockIdx.x * IT + it) * W;
      if (u0 >= nunits) break;  // uniform
      units(u0);
    }
  }
}

// I2 of the scaled grids: the y columns (level row z, kx) of the z pass's
// folded output, folded along y to length P and inverted, rows y < N kept:
// A[z][y][kx] (kx < S P / 2, the x half spectrum).
template <class R, int P, int S>
__global__ void __launch_bounds__((Cfg<R, P, kPassIY>::WS * Cfg<R, P, kPassIY>::TL), (Cfg<R, P, kPassIY>::MINW))
k_inv_y_fold(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassIY>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WS, PS = S * P, HS = PS / 2, NT = HS / W;
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw[P];
  const TwStage<R, P, C::WS * C::TL, S> tws(tb.tw);  // tb: the period-S P tables
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = g.N;
  const int z = blockIdx.x / NT;
  if (z >= N) return;  // uniform: a smaller grid of a mixed launch
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int kx = (blockIdx.x % NT) * W + w;
  const T* B0 = static_cast<const T*>(F.B) + (size_t)z * zrow_pitch(PS, sizeof(T)) + kx;  // ky at + ky HS
  T v[E];
#pragma unroll
  for (int q = 0; q < E; ++q)
    v[q] = fold_to_p<R, P, S>([&](int ky) { return B0[(size_t)ky * HS]; }, t + TL * q, tb.tw);
  LdsView<R> lds{sre, sim, W, 1, w};
  tws.put(stw);
  fft_line<R, P, +1, false, true, kPassIY>(v, t, lds, stw);
  T* A = static_cast<T*>(F.A) + (size_t)z * N * HS + kx;
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int y = t + TL * q;
    if (y < N) A[(size_t)y * HS] = v[q];
  }
}

// Out(x) of the row `orow` plus the reduced scaled-grid value m and, when
// S is set, Prolong(S_{l-1}); TwoSum on the compensated FP32 path.  For a
// doubled grid out holds the hole potential, for a quadrupled grid (run
// after it) the sum so far.
template <class R, bool TRI>
__device__ __forceinline__ void scaled_out(const FieldDesc& F, R* orow, const R* S, const R* Sl,
                                           const CarryRows& cr, int x, R m) {
  const R base = orow[x];
  R hi, lo = 0;
  if (sizeof(R) == 8 || !F.comp) {
    hi = base + m;
    if (S) {
      R s1, l;
      carried<R, TRI>(F.comp, S, Sl, cr, x, s1, l);
      hi += s1;
    }
  } else {
    two_sum(base, m, hi, lo);
    if (S) {
      R s1, l, s2, e3;
      carried<R, TRI>(F.comp, S, Sl, cr, x, s1, l);
      two_sum(hi, s1, s2, e3);
      hi = s2;
      lo += e3 + l;
    }
  }
  orow[x] = hi + lo;
}

// I1 of the scaled grids: the x half spectra (period S P) of level rows
// (z, y) and (z, y + 1), folded to the packed half spectra of length P and
// inverted as one complex transform (row y in the real part, y + 1 in the
// imaginary part); the S^3 means are added to out (scaled_out).
template <class R, int P, int S, bool TRI>
__global__ void __launch_bounds__((Cfg<R, P, kPassIX>::WC * Cfg<R, P, kPassIX>::TL))
k_inv_x_fold(FieldTable ft, PassGeom g, Tables<R> tb) {
  using C = Cfg<R, P, kPassIX>;
  using T = cplx<R>;
  constexpr int E = C::E, TL = C::TL, W = C::WC, PS = S * P, HS = PS / 2;
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw[P];
  const TwStage<R, P, C::WC * C::TL, S> tws(tb.tw);  // tb: the period-S P tables
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = g.N;
  const int nunits = N * N / 2;
  if ((int)blockIdx.x * W >= nunits) return;  // uniform: a smaller grid of a mixed launch
  const int t = threadIdx.x % TL, w = threadIdx.x / TL;
  const int unit = blockIdx.x * W + w;
  const bool active = unit < nunits;
  const int line = active ? 2 * unit : 0;
  const int z = line / N, y = line % N;
  const T* ra = static_cast<const T*>(F.A) + ((size_t)z * N + y) * HS;
  const T* rb = ra + HS;
  // X[m], 0 <= m < S P, of a real line from its packed half spectrum
  // (slot 0: the real DC and Nyquist values; X[S P - m] = conj X[m])
  auto spec = [](const T* r, int m) -> T {
    const int i = m <= HS ? m : PS - m;
    const T a = r[i == HS ? 0 : i];
    const T u = i == 0 ? T{a.x, 0} : i == HS ? T{a.y, 0} : a;
    return m <= HS ? u : T{u.x, -u.y};
  };
  // Y[k], 0 <= k <= P/2; Y[0] and Y[P/2] are real
  auto folded = [&](const T* r, int k) -> T {
    const T u = fold_to_p<R, P, S>([&](int m) { return spec(r, m); }, k, tb.tw);
    return (k == 0 || k == P / 2) ? T{u.x, 0} : u;
  };
  T v[E];
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int k = t + TL * q;  // < P/2
    const T a = folded(ra, k), b = folded(rb, k);
    v[q] = active ? T{a.x - b.y, a.y + b.x} : T{0, 0};
  }
#pragma unroll
  for (int q = E / 2; q < E; ++q) {
    const int kk = P - (t + TL * q);  // in (0, P/2]
    const T a = folded(ra, kk), b = folded(rb, kk);
    v[q] = active ? T{a.x + b.y, b.x - a.y} : T{0, 0};  // conj(Y_a) + i conj(Y_b)
  }
  LdsView<R> lds{sre, sim, 1, P, w};
  tws.put(stw);
  fft_line<R, P, +1, false, true, kPassIX>(v, t, lds, stw);
  if (!active) return;
  const int NS = N / 2 + 2;
  R* out = static_cast<R*>(F.out);
  const R* Sc = static_cast<const R*>(F.S);
  const R* Sl = static_cast<const R*>(F.Slo);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int yy = y + h;
    const CarryRows cr = carry_rows(z, yy, NS);
    R* orow = out + ((size_t)z * N + yy) * N;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int x = t + TL * q;
      if (x < N) scaled_out<R, TRI>(F, orow, Sc, Sl, cr, x, h == 0 ? v[q].x : v[q].y);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused plane passes (P <= 64): a workgroup owns one z plane of one grid and
// keeps it in LDS between the x and y transforms, so the x-transformed plane
// never goes through HBM and one launch does the work of two.  (Measured: at
// P = 128 the one-workgroup-per-plane grid, e.g. 576 workgroups for 9 grids
// of 64^3, leaves too little parallelism and the separate passes win.)
//   XY  (fwd_xy): the x lines of the plane (as the X pass), then its y
//                 columns (as the Y pass), written to B[z][ky][kx];
//   IYX (inv_yx): the y columns of an output plane (as the I2 pass), then its
//                 x lines (as the I1 pass, with the same outputs and carry).
#ifndef NMC_PLANE_THREADS
#define NMC_PLANE_THREADS 256
#endif
template <class R, int P>
struct PlaneCfg {
  static constexpr int E = Plan<R, P, kPassOther>::E;
  static constexpr int TL = P / E;
  static constexpr int H2 = P / 2;
  static constexpr int WL = (NMC_PLANE_THREADS / TL < H2) ? NMC_PLANE_THREADS / TL : H2;  // lines per round
  static constexpr int NTH = WL * TL;
  static constexpr int PS = H2 + 1;  // plane row stride: odd, so column reads spread over banks
  static constexpr int LDS = (2 * H2 * PS + 2 * WL * P) * (int)sizeof(R) + P * 2 * (int)sizeof(R);
};
constexpr int kPlaneLdsMax = 64 * 1024;
constexpr int kPlaneMaxP = 64;

template <class R, int P, bool FULLN>
__global__ void __launch_bounds__((PlaneCfg<R, P>::NTH)) k_fwd_xy(FieldTable ft, PassGeom g, Tables<R> tb) {
  using PC = PlaneCfg<R, P>;
  using T = cplx<R>;
  constexpr int E = PC::E, TL = PC::TL, WL = PC::WL, PS = PC::PS, H2 = PC::H2;
  __shared__ R pre[H2 * PS], pim[H2 * PS];
  __shared__ R sre[WL * P], sim[WL * P];
  __shared__ T stw[P];
  const TwStage<R, P, PC::NTH> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = FULLN ? P / 2 : g.N;
  const int n = grid_geo(F.kind, N).nin;
  const int z = blockIdx.x;
  if (z >= n) return;  // uniform: a smaller grid of a mixed launch
  tws.put(stw);
  {  // x lines y of the plane, t fastest (rows of the density are contiguous)
    const int t = threadIdx.x % TL, w = threadIdx.x / TL;
    const LdsView<R> lds{sre, sim, 1, P, w};
    // the next round's inputs are loaded while this round is transformed
    T vn[E];
    x_inputs<R, P, FULLN, kPassOther>(F, N, z, w < n ? w : 0, w < n, t, vn);
    for (int y0 = 0; y0 < n; y0 += WL) {
      const int y = y0 + w;
      const bool active = y < n;
      T v[E];
#pragma unroll
      for (int q = 0; q < E / 2; ++q) v[q] = vn[q];
      if (y0 + WL < n) {  // uniform
        const int yn = y + WL;
        x_inputs<R, P, FULLN, kPassOther>(F, N, z, yn < n ? yn : 0, yn < n, t, vn);
      }
      fft_line<R, P, -1, true, false, kPassOther>(v, t, lds, stw);
      if (active) {
#pragma unroll
        for (int q = 0; q < E / 2; ++q) {
          const T o = x_packed<R, P, kPassOther>(v, t, q);
          pre[y * PS + t + TL * q] = o.x;
          pim[y * PS + t + TL * q] = o.y;
        }
      }
    }
  }
  __syncthreads();
  {  // y columns kx, w fastest (each store is a run of WL complex values)
    const int w = threadIdx.x % WL, t = threadIdx.x / WL;
    const LdsView<R> lds{sre, sim, WL, 1, w};
    const bool full_in = FULLN && F.kind != 1;
    T* Bz = static_cast<T*>(F.B) + (size_t)z * zrow_pitch(P, sizeof(T));
    for (int k0 = 0; k0 < H2; k0 += WL) {
      const int kx = k0 + w;
      T v[E];
#pragma unroll
      for (int q = 0; q < E / 2; ++q) {
        const int yy = t + TL * q;
        v[q] = (full_in || yy < n) ? T{pre[yy * PS + kx], pim[yy * PS + kx]} : T{0, 0};
      }
      fft_line<R, P, -1, true, false, kPassOther>(v, t, lds, stw);
#pragma unroll
      for (int q = 0; q < E; ++q) Bz[(size_t)(t + TL * q) * H2 + kx] = v[q];
    }
  }
}

template <class R, int P, bool FULLN, bool TRI>
__global__ void __launch_bounds__((PlaneCfg<R, P>::NTH)) k_inv_yx(FieldTable ft, PassGeom g, Tables<R> tb) {
  using PC = PlaneCfg<R, P>;
  using T = cplx<R>;
  constexpr int E = PC::E, TL = PC::TL, WL = PC::WL, PS = PC::PS, H2 = PC::H2;
  __shared__ R pre[H2 * PS], pim[H2 * PS];
  __shared__ R sre[WL * P], sim[WL * P];
  __shared__ T stw[P];
  const TwStage<R, P, PC::NTH> tws(tb.tw);
  const FieldDesc& F = ft.f[blockIdx.y];
  const int N = FULLN ? P / 2 : g.N;
  const GridGeo gg = grid_geo(F.kind, N);
  const int n = gg.nout;
  const int zr = blockIdx.x;
  if (zr >= n) return;  // uniform: a smaller grid of a mixed launch
  const int z = gg.olo + zr;
  tws.put(stw);
  {  // y columns kx: inverse, keep the output rows [olo, olo + n)
    const int w = threadIdx.x % WL, t = threadIdx.x / WL;
    const LdsView<R> lds{sre, sim, WL, 1, w};
    const T* Bz = static_cast<const T*>(F.B) + (size_t)z * zrow_pitch(P, sizeof(T));
    // the next round's columns are loaded while this round is transformed
    T vn[E];
#pragma unroll
    for (int q = 0; q < E; ++q) vn[q] = Bz[(size_t)(t + TL * q) * H2 + w];
    for (int k0 = 0; k0 < H2; k0 += WL) {
      const int kx = k0 + w;
      T v[E];
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = vn[q];
      if (k0 + WL < H2) {  // uniform
#pragma unroll
        for (int q = 0; q < E; ++q) vn[q] = Bz[(size_t)(t + TL * q) * H2 + kx + WL];
      }
      fft_line<R, P, +1, false, true, kPassOther>(v, t, lds, stw);
#pragma unroll
      for (int q = 0; q < E / 2; ++q) {
        const int yr = t + TL * q - gg.olo;
        if (yr >= 0 && yr < n) {
          pre[yr * PS + kx] = v[q].x;
          pim[yr * PS + kx] = v[q].y;
        }
      }
    }
  }
  __syncthreads();
  {  // x lines of the output rows: C2R, then the outputs of the I1 pass
    const int t = threadIdx.x % TL, w = threadIdx.x / TL;
    const LdsView<R> lds{sre, sim, 1, P, w};
    for (int y0 = 0; y0 < n; y0 += WL) {
      const int yr = y0 + w;
      const bool active = yr < n;
      const int yc = active ? yr : 0;
      T v[E];
      hermitian_inputs<R, P, kPassOther>([&](int k) { return T{pre[yc * PS + k], pim[yc * PS + k]}; }, active, t, v);
      fft_line<R, P, +1, false, true, kPassOther>(v, t, lds, stw);
      if (active) ix_outputs<R, P, kPassOther, TRI>(F, N, gg, z, gg.olo + yr, zr, yr, t, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Restriction: mean of the 2^3 children of every child-region cell.
template <class R>
__global__ void k_restrict(const R* __restrict__ fine, const R* __restrict__ fine_rc,
                           R* __restrict__ rc, int N) {
  const int N2 = N / 2, lo = N / 4, hi = 3 * N / 4;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N2 * N2 * N2) return;
  const int ax = id % N2, ay = (id / N2) % N2, az = id / (N2 * N2);
  R s = 0;
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int z = 2 * az + bz, y = 2 * ay + by, x = 2 * ax + bx;
        const bool cen = fine_rc && z >= lo && z < hi && y >= lo && y < hi && x >= lo && x < hi;
        s += cen ? fine_rc[((size_t)(z - lo) * N2 + (y - lo)) * N2 + (x - lo)]
                 : fine[((size_t)z * N + y) * N + x];
      }
  rc[id] = s * (R)0.125;
}

// Block-mean pyramids (the unrolled restriction, kernels.h).  A workgroup
// owns an aligned cube of S = pyramid_cube(N, k) cells per axis of one
// level k >= 1: every thread forms the 2x2x2 means of m_k (the density with
// the level's child region zeroed, except on the finest level) of its
// sub-blocks, all loads issued together, then the means of those means up
// to blocks of 2^k cells are formed in LDS, every size written to the
// level's slab.
constexpr int kPyramidThreads = 512;
template <class R>
__global__ void __launch_bounds__(kPyramidThreads) k_pyramid(PyramidTable tab, int N, int maxL) {
  using T2 = cplx<R>;
  const PyramidDesc& D = tab.r[blockIdx.y];
  int b = blockIdx.x, k = 1, S = 0, nc = 0;
  for (; k < maxL; ++k) {
    S = pyramid_cube(N, k);
    nc = N / S;
    if (b < nc * nc * nc) break;
    b -= nc * nc * nc;
  }
  if (k >= D.L) return;  // uniform: a request with fewer levels
  const R* rho = static_cast<const R*>(D.rho) + (size_t)k * N * N * N;
  R* pyr = static_cast<R*>(D.pyr) + (size_t)(k - 1) * D.slab;
  const int ox = (b % nc) * S, oy = (b / nc % nc) * S, oz = b / (nc * nc) * S;
  const bool mask = k < D.L - 1;
  const int lo = N / 4, hi = 3 * N / 4;
  constexpr int S0 = 1 << kMaxPyramidDepth;
  constexpr int NSUB = (S0 / 2) * (S0 / 2) * (S0 / 2);
  constexpr int IT = NSUB / kPyramidThreads;  // sub-blocks per thread at the largest cube
  __shared__ R buf[NSUB + (S0 / 4) * (S0 / 4) * (S0 / 4)];
  R* src = buf;
  R* dst = buf + NSUB;
  int e = S / 2;  // blocks per axis of the cube at the current size
  const int ne = e * e * e;
  {
    // x pairs (even x) as one vector load; a masked cell or a thread past
    // the cube reads a valid pair and drops it
    T2 val[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      if (it * kPyramidThreads >= ne) break;  // uniform
      const int j = min((int)threadIdx.x + it * kPyramidThreads, ne - 1);
      const int gx = ox + 2 * (j % e), gy = oy + 2 * (j / e % e), gz = oz + 2 * (j / (e * e));
#pragma unroll
      for (int a = 0; a < 4; ++a)
        val[it][a] = *reinterpret_cast<const T2*>(rho + ((size_t)(gz + (a >> 1)) * N + gy + (a & 1)) * N + gx);
    }
    const int nd = N >> 1;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int j = (int)threadIdx.x + it * kPyramidThreads;
      if (j >= ne) break;
      const int gx = ox + 2 * (j % e), gy = oy + 2 * (j / e % e), gz = oz + 2 * (j / (e * e));
      R s = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int zz = gz + (a >> 1), yy = gy + (a & 1);
        const bool yz_in = mask && zz >= lo && zz < hi && yy >= lo && yy < hi;
        if (!(yz_in && gx >= lo && gx < hi)) s += val[it][a].x;
        if (!(yz_in && gx + 1 >= lo && gx + 1 < hi)) s += val[it][a].y;
      }
      const R m = s * (R)0.125;
      pyr[((size_t)(gz >> 1) * nd + (gy >> 1)) * nd + (gx >> 1)] = m;
      if (k >= 2) src[j] = m;
    }
  }
  size_t off = (size_t)(N >> 1) * (N >> 1) * (N >> 1);
  for (int d = 2; d <= k; ++d) {
    __syncthreads();
    const int e2 = e / 2, nd = N >> d;
    for (int j = threadIdx.x; j < e2 * e2 * e2; j += blockDim.x) {
      const int sx = j % e2, sy = j / e2 % e2, sz = j / (e2 * e2);
      R s = 0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int x = 0; x < 2; ++x) s += src[((2 * sz + a) * e + 2 * sy + c) * e + 2 * sx + x];
      const R m = s * (R)0.125;
      pyr[off + ((size_t)((oz >> d) + sz) * nd + (oy >> d) + sy) * nd + (ox >> d) + sx] = m;
      dst[j] = m;
    }
    R* t = src;
    src = dst;
    dst = t;
    e = e2;
    off += (size_t)nd * nd * nd;
  }
}

// One step of the carry cascade, S = (3/4 A + 1/4 B) + Phi_hole (the diagonal
// rule of Eqs. 3-6); with comp, (hi, lo) pairs carry the rounding error of
// every operation (TwoSum, and an FMA for the product by 3/4).
template <class R, bool COMP>
__device__ __forceinline__ void carry_step(R ahi, R alo, R bhi, R blo, R h, R& hi, R& lo) {
  if constexpr (sizeof(R) == 8 || !COMP) {
    hi = ((R)0.75 * ahi + (R)0.25 * bhi) + h;
    lo = 0;
  } else {
    const R p1 = (R)0.75 * ahi;
    const R e1 = fma((R)0.75, ahi, -p1);
    R s, e2;
    two_sum(p1, (R)0.25 * bhi, s, e2);
    R l = e1 + e2;
    l += (R)0.75 * alo + (R)0.25 * blo;
    R s2, e3;
    two_sum(s, h, s2, e3);
    l += e3;
    hi = s2 + l;  // renormalise
    lo = l - (hi - s2);
  }
}

// S_n at box cell (bz, by, bx), unrolling D steps of the cascade down to
// S_{n-D}, read from (lhi, llo) (llo null: no compensation term).  Box cell
// b is level cell b + N/4 - 1; a fine cell f takes its parent f/2 + 1 (box
// coordinates of the coarser level) and the diagonal neighbour one further
// in every axis, towards f's side of the parent.  D is a compile-time depth
// so that every load of the tree is issued before the first is used.
template <class R, bool COMP, int D>
__device__ __forceinline__ void carry_tree(const CarryDesc& C, int N, int n, const R* lhi, const R* llo,
                                           int bz, int by, int bx, R& hi, R& lo) {
  const int NB = N / 2 + 2;
  const size_t id = ((size_t)bz * NB + by) * NB + bx;
  if constexpr (D == 0) {
    hi = lhi[id];
    const R l = (llo ? llo : lhi)[id];  // no branch around the load
    lo = llo ? l : (R)0;
  } else {
    const int off = N / 4 - 1;
    const int z = bz + off, y = by + off, x = bx + off;
    const int iz = z / 2 + 1, iy = y / 2 + 1, ix = x / 2 + 1;
    R ahi, alo, bhi, blo;
    carry_tree<R, COMP, D - 1>(C, N, n - 1, lhi, llo, iz, iy, ix, ahi, alo);
    carry_tree<R, COMP, D - 1>(C, N, n - 1, lhi, llo, iz + ((z & 1) ? 1 : -1), iy + ((y & 1) ? 1 : -1),
                               ix + ((x & 1) ? 1 : -1), bhi, blo);
    const R h = static_cast<const R*>(C.hole)[(size_t)n * C.box + id];
    carry_step<R, COMP>(ahi, alo, bhi, blo, h, hi, lo);
  }
}

// COMP: every request of the launch keeps (hi, lo) pairs (CarryDesc::comp).
template <class R, bool COMP>
__global__ void __launch_bounds__(256) k_carry(CarryTable tab, int N, int n0) {
  const int NB = N / 2 + 2, nb3 = NB * NB * NB, per = (nb3 + 255) / 256;
  const int r = blockIdx.y, lv = blockIdx.x / per;
  if (lv >= tab.nlev[r]) return;  // uniform: a request with fewer levels
  const int id = (blockIdx.x % per) * 256 + threadIdx.x;
  if (id >= nb3) return;
  const CarryDesc& C = tab.r[r];
  const int n = n0 + lv;
  // S_{n0-1}: the hole potential of level 0 itself when n0 = 1
  const R* S = static_cast<const R*>(C.S);
  const R* lhi = n0 == 1 ? static_cast<const R*>(C.hole) : S + (size_t)(n0 - 1) * 2 * C.box;
  const R* llo = (n0 == 1 || !COMP) ? nullptr : lhi + C.box;
  const int bz = id / (NB * NB), by = id / NB % NB, bx = id % NB;
  R hi, lo;
  static_assert(kMaxCarryDepth == 4, "one case per depth");
  switch (lv) {
    case 0: carry_tree<R, COMP, 1>(C, N, n, lhi, llo, bz, by, bx, hi, lo); break;
    case 1: carry_tree<R, COMP, 2>(C, N, n, lhi, llo, bz, by, bx, hi, lo); break;
    case 2: carry_tree<R, COMP, 3>(C, N, n, lhi, llo, bz, by, bx, hi, lo); break;
    default: carry_tree<R, COMP, 4>(C, N, n, lhi, llo, bz, by, bx, hi, lo); break;
  }
  R* out = static_cast<R*>(C.S) + (size_t)n * 2 * C.box;
  out[id] = hi;
  if (COMP) out[C.box + id] = lo;
}

// One level n of the carry cascade with the tensor-product rule
// (NMC_PROLONG_TRILINEAR): S_n = Prolong(S_{n-1}) + Phi^n_hole on the
// stencil box, S_0 = Phi^0_hole.  Each S_n reads 8 values of S_{n-1}, so the
// cascade is not unrolled (one launch per level).
template <class R, bool COMP>
__global__ void __launch_bounds__(256) k_carry_tri(CarryTable tab, int N, int n) {
  const int NB = N / 2 + 2, nb3 = NB * NB * NB;
  const int r = blockIdx.y;
  if (n > tab.nlev[r]) return;  // uniform: a request with fewer levels
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= nb3) return;
  const CarryDesc& C = tab.r[r];
  const R* S = static_cast<const R*>(C.S);
  const R* phi = n == 1 ? static_cast<const R*>(C.hole) : S + (size_t)(n - 1) * 2 * C.box;
  const R* plo = (n == 1 || !COMP) ? nullptr : phi + C.box;
  const int off = N / 4 - 1;  // box cell b is level cell b + off
  const int bz = id / (NB * NB), by = id / NB % NB, bx = id % NB;
  R s, l, hi, lo = 0;
  carried<R, true>(COMP, phi, plo, carry_rows(bz + off, by + off, NB), bx + off, s, l);
  const R h = static_cast<const R*>(C.hole)[(size_t)n * C.box + id];
  if constexpr (sizeof(R) == 8 || !COMP) {
    hi = s + h;
  } else {
    R e;
    two_sum(s, h, hi, e);
    lo = e + l;
  }
  R* out = static_cast<R*>(C.S) + (size_t)n * 2 * C.box;
  out[id] = hi;
  if (COMP) out[C.box + id] = lo;
}

// ---------------------------------------------------------------------------
// Gravitational acceleration g = -grad Phi on every level (Sect. 2, the
// six-point central stencil), with the rules of Appendix A next to the
// coarse-fine interfaces: a neighbour outside the level (level >= 1) is the
// boundary value interpolated from the coarser level by Eqs. 3-6, diagonal
// 3/4-1/4 rule (method A); a neighbour inside the child region of a cell
// outside it takes the mean of the finer level's potential over the 2^3
// cells it covers (method B).  The coarsest level's outer faces use the
// second-order one-sided difference; covered cells use the level's own
// values.  One thread per cell (blocks: runs of a z plane), all three
// components.
template <class R>
__device__ __forceinline__ R accel_neighbour(const R* __restrict__ P, const R* __restrict__ Pc,
                                             const R* __restrict__ Pf, int N, int z, int y, int x,
                                             bool centre_in) {
  const int lo = N / 4, hi = 3 * N / 4;
  const bool in_level = (unsigned)z < (unsigned)N && (unsigned)y < (unsigned)N && (unsigned)x < (unsigned)N;
  if (!in_level) {  // method A (the caller never asks on the coarsest level)
    auto par = [&](int f) { return N / 4 + (f >= 0 ? f / 2 : -1); };  // N/4 + floor(f/2), f >= -1
    auto sgn = [&](int f) { return (f & 1) ? 1 : -1; };
    const int cz = par(z), cy = par(y), cx = par(x);
    const R a = Pc[((size_t)cz * N + cy) * N + cx];
    const R b = Pc[((size_t)(cz + sgn(z)) * N + (cy + sgn(y))) * N + (cx + sgn(x))];
    return (R)0.75 * a + (R)0.25 * b;
  }
  const bool n_in = z >= lo && z < hi && y >= lo && y < hi && x >= lo && x < hi;
  if (Pf && n_in && !centre_in) {  // method B
    const int fz = 2 * (z - lo), fy = 2 * (y - lo), fx = 2 * (x - lo);
    R s = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) s += Pf[((size_t)(fz + a) * N + (fy + b)) * N + (fx + c)];
    return s * (R)0.125;
  }
  return P[((size_t)z * N + y) * N + x];
}

template <class R>
__global__ void __launch_bounds__(256) k_accel(const R* __restrict__ phi, R* __restrict__ g, int N, int L,
                                               double h0) {
  const size_t n3 = (size_t)N * N * N;
  const int l = blockIdx.z, z = blockIdx.y;
  const int col = blockIdx.x * 256 + threadIdx.x;  // 32-bit: no 64-bit division
  if (col >= N * N) return;
  const int x = col % N, y = col / N;
  const size_t id = (size_t)z * N * N + col;
  const R* P = phi + (size_t)l * n3;
  const R* Pc = l > 0 ? P - n3 : nullptr;
  const R* Pf = l + 1 < L ? P + n3 : nullptr;
  const int lo = N / 4, hi = 3 * N / 4;
  const bool centre_in = z >= lo && z < hi && y >= lo && y < hi && x >= lo && x < hi;
  const R h = (R)ldexp(h0, -l);
  const R inv2h = (R)1 / (2 * h);
  const int c[3] = {x, y, z};
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    const int i = c[comp];
    R gv;
    if (l == 0 && (i == 0 || i == N - 1)) {  // coarsest outer face: one-sided
      const int d = i == 0 ? 1 : -1;
      int q1[3] = {x, y, z}, q2[3] = {x, y, z};
      q1[comp] += d;
      q2[comp] += 2 * d;
      const R p0 = P[id];
      const R p1 = P[((size_t)q1[2] * N + q1[1]) * N + q1[0]];
      const R p2 = P[((size_t)q2[2] * N + q2[1]) * N + q2[0]];
      gv = -(R)d * ((R)-3 * p0 + (R)4 * p1 - p2) * inv2h;
    } else {
      int qp[3] = {x, y, z}, qm[3] = {x, y, z};
      qp[comp] += 1;
      qm[comp] -= 1;
      const R vp = accel_neighbour(P, Pc, Pf, N, qp[2], qp[1], qp[0], centre_in);
      const R vm = accel_neighbour(P, Pc, Pf, N, qm[2], qm[1], qm[0], centre_in);
      gv = -(vp - vm) * inv2h;
    }
    g[((size_t)l * 3 + comp) * n3 + id] = gv;
  }
}

// ---------------------------------------------------------------------------
// Green spectrum, FP64.  The kernel on the doubled mesh is even in every
// axis, so its transform is real and even and separable passes over the
// octant [0, P/2]^3 suffice: each line of P values is rebuilt by even
// extension, transformed, and the real parts of k = 0..P/2 are kept.
template <int P>
__global__ void __launch_bounds__((Cfg<double, P, kPassOther>::WC * Cfg<double, P, kPassOther>::TL))
k_green(int pass, double beta, const double2* tw, const double* __restrict__ src,
        double* __restrict__ dst) {
  using C = Cfg<double, P, kPassOther>;
  constexpr int E = C::E, TL = C::TL, W = C::WC, H = P / 2 + 1;
  __shared__ double sre[W * P], sim[W * P];
  __shared__ double2 stw[P];
  stage_twiddles<double, P>(stw, tw);
  const int t = threadIdx.x % TL, w = threadIdx.x / TL;
  const int line = blockIdx.x * W + w;
  const bool active = line < H * H;
  const int a = active ? line % H : 0, b = active ? line / H : 0;
  double2 v[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int n = t + TL * q;
    const int d = n <= P / 2 ? n : P - n;
    double val = 0;
    if (active) {
      if (pass == 0) {
        const double r2 = (double)d * d + (double)a * a + (double)b * b;
        val = r2 == 0 ? beta : 1.0 / sqrt(r2);
      } else if (pass == 1) {
        val = src[((size_t)b * H + d) * H + a];
      } else {
        val = src[((size_t)d * H + b) * H + a];
      }
    }
    v[q] = double2{val, 0};
  }
  LdsView<double> lds{sre, sim, 1, P, w};
  fft_line<double, P, -1, false, false, kPassOther>(v, t, lds, stw);
  if (!active) return;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int k = t + TL * q;
    if (k <= P / 2) {
      size_t o;
      if (pass == 0) o = ((size_t)b * H + a) * H + k;
      else if (pass == 1) o = ((size_t)b * H + k) * H + a;
      else o = ((size_t)k * H + b) * H + a;
      dst[o] = v[q].x;
    }
  }
}

__global__ void k_round_f32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// Reorder the octant [kz][ky][kx] into gz[kyp][tile][kzp][w] and gn[kyp][kzp].
template <class R, int P>
__global__ void k_green_layout(const double* __restrict__ oct, R* __restrict__ gz, R* __restrict__ gn) {
  constexpr int H = P / 2 + 1, W = Cfg<R, P, kPassZ>::WZ, NT = (P / 2) / W;
  const size_t n = (size_t)H * NT * H * W;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int w = i % W, kzp = (i / W) % H, tile = (i / ((size_t)W * H)) % NT, kyp = i / ((size_t)W * H * NT);
    gz[i] = (R)oct[((size_t)kzp * H + kyp) * H + tile * W + w];
  }
  if (i < (size_t)H * H) {
    const int kzp = i % H, kyp = i / H;
    gn[i] = (R)oct[((size_t)kzp * H + kyp) * H + P / 2];
  }
}

// Diagnostic: batched unpruned 1-D FFT of contiguous lines.
template <class R, int P, int DIR>
__global__ void __launch_bounds__((Cfg<R, P, kPassOther>::WC * Cfg<R, P, kPassOther>::TL))
k_fft_lines(const cplx<R>* __restrict__ in, cplx<R>* __restrict__ out, int nlines,
            const cplx<R>* tw) {
  using C = Cfg<R, P, kPassOther>;
  constexpr int E = C::E, TL = C::TL, W = C::WC;
  __shared__ R sre[W * P], sim[W * P];
  __shared__ cplx<R> stw[P];
  stage_twiddles<R, P>(stw, tw);
  const int t = threadIdx.x % TL, w = threadIdx.x / TL;
  const int line = blockIdx.x * W + w;
  const bool active = line < nlines;
  cplx<R> v[E];
#pragma unroll
  for (int q = 0; q < E; ++q)
    v[q] = active ? in[(size_t)line * P + t + TL * q] : cplx<R>{0, 0};
  LdsView<R> lds{sre, sim, 1, P, w};
  fft_line<R, P, DIR, false, false, kPassOther>(v, t, lds, stw);
  if (!active) return;
#pragma unroll
  for (int q = 0; q < E; ++q) out[(size_t)line * P + t + TL * q] = v[q];
}

// ---------------------------------------------------------------------------
// Host launchers.

namespace {
thread_local hipEvent_t g_next_start = nullptr, g_next_stop = nullptr;
}
void set_next_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_next_start = start;
  g_next_stop = stop;
}
bool take_next_launch_events() {
  const bool pending = g_next_start != nullptr;
  g_next_start = g_next_stop = nullptr;
  return pending;
}
// hipLaunchKernelGGL, with the pending timing events if any
template <class K, class... Args>
static void launch(K kernel, dim3 grid, dim3 block, unsigned shmem, hipStream_t s, Args... args) {
  hipEvent_t a = g_next_start, b = g_next_stop;
  g_next_start = g_next_stop = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, args...);
}

// Periods up to MAXP: 512 for level grids (N <= 256), 1024 where a scaled
// grid of the modified methods can need it (doubled grids of N = 256,
// quadrupled grids of N = 128) and for the Green tables of that period.
template <int MAXP = 512, class F>
static hipError_t dispatch_p(int P, F&& f) {
  switch (P) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024:
      if constexpr (MAXP >= 1024) {
        f(std::integral_constant<int, 1024>{});
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Line pairs per transform in the x passes: not for FP32 below N = 128 (there
// the twice larger grid of single-line workgroups measured faster).
template <class R>
bool x_pairs(int N) {
  return sizeof(R) == 8 || N >= 128;
}

template <class R>
hipError_t launch_fwd_x(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  const bool pairs = x_pairs<R>(g.N);
  return dispatch_p<1024>(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassX>;
    const int units = pairs ? g.n * g.n / 2 : g.n * g.n;
    constexpr int UW = C::WC * x_iters<PP>();  // units per workgroup
    dim3 grid((units + UW - 1) / UW, g.nf), block(C::WC * C::TL);
    const bool full = g.N == PP / 2;
    if constexpr (PP >= 16) {
      if (PP >= 4 * g.N) {  // scaled grids
        if (pairs) launch(k_fwd_x<R, PP, false, true, true>, grid, block, 0, s, ft, g, tb);
        else launch(k_fwd_x<R, PP, false, false, true>, grid, block, 0, s, ft, g, tb);
        return;
      }
    }
    if constexpr (PP > 512) return;  // level grids stop at 512 (the runtime checks)
    else if (pairs && full) launch(k_fwd_x<R, PP, true, true>, grid, block, 0, s, ft, g, tb);
    else if (pairs) launch(k_fwd_x<R, PP, false, true>, grid, block, 0, s, ft, g, tb);
    else if (full) launch(k_fwd_x<R, PP, true, false>, grid, block, 0, s, ft, g, tb);
    else launch(k_fwd_x<R, PP, false, false>, grid, block, 0, s, ft, g, tb);
  });
}

template <class R>
hipError_t launch_fwd_y(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  return dispatch_p<1024>(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassY>;
    dim3 grid(((PP / 2) / C::WS) * g.n, g.nf);
    if constexpr (PP >= 16) {
      if (PP >= 4 * g.N) {  // scaled grids
        launch(k_fwd_y<R, PP, false, true>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
        return;
      }
    }
    if constexpr (PP > 512) return;  // level grids stop at 512
    else if (g.N == PP / 2)
      launch(k_fwd_y<R, PP, true>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
    else
      launch(k_fwd_y<R, PP, false>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
  });
}

template <class R>
hipError_t launch_z(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  return dispatch_p<1024>(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassZ>;
    constexpr int NT = (PP / 2) / C::WZ;
    dim3 grid(NT * (PP / 2) * g.nf);  // one dimension: see k_z, z_unit
    if (PP >= 4 * g.N) {  // scaled grids
      using CS = Cfg<R, PP, kPassZScaled>;
      const dim3 block(2 * CS::WZ * CS::TL);
      static_assert(z_col0_split<R, PP, 2>() == z_col0_split<R, PP, 4>(), "one grid size for both scales");
      if constexpr (PP == 1024 && NMC_Z_ONE_ROW_SCALED) {
        // one-row workgroups of 2 W columns, column 0 apart
        const dim3 g1(z_col0_blocks(NT, g.nf) + (PP / 2) / (2 * C::WZ) * PP * g.nf);
        if (g.S == 2) launch(k_z<R, PP, false, 2, true>, g1, block, 0, s, ft, g, tb);
        else if (g.S == 4) launch(k_z<R, PP, false, 4, true>, g1, block, 0, s, ft, g, tb);
        return;
      }
      if constexpr (z_col0_split<R, PP, 2>()) grid.x += z_col0_blocks(NT, g.nf);
      if constexpr (PP >= 16) {
        if (g.S == 2) launch(k_z<R, PP, false, 2>, grid, block, 0, s, ft, g, tb);
      }
      if constexpr (PP >= 32) {
        if (g.S == 4) launch(k_z<R, PP, false, 4>, grid, block, 0, s, ft, g, tb);
      }
      return;
    }
    if constexpr (PP <= 512) {  // level grids stop at 512 (the runtime checks)
      if constexpr (PP == 512 && sizeof(R) == 4 && NMC_Z_STAGED) {  // FP32 (FP64: k_z measured faster)
        using G = zs::Geo<R>;
        const dim3 gs((G::UNITS + PP / 2) * g.nf), bs(G::NT);
        if (g.N == PP / 2)
          launch(k_zs<R, true>, gs, bs, 0, s, ft, g, tb);
        else
          launch(k_zs<R, false>, gs, bs, 0, s, ft, g, tb);
        return;
      }
      if constexpr (PP == 512 && NMC_Z_ONE_ROW && (sizeof(R) == 8 || NMC_Z_ONE_ROW_F32)) {
        // one-row workgroups of 2 W columns (128-byte runs), column 0 apart
        const dim3 g1(z_col0_blocks(NT, g.nf) + (PP / 2) / (2 * C::WZ) * PP * g.nf);
        if (g.N == PP / 2)
          launch(k_z<R, PP, true, 1, true>, g1, dim3(2 * C::WZ * C::TL), 0, s, ft, g, tb);
        else
          launch(k_z<R, PP, false, 1, true>, g1, dim3(2 * C::WZ * C::TL), 0, s, ft, g, tb);
        return;
      }
      if constexpr (z_col0_split<R, PP, 1>()) grid.x += z_col0_blocks(NT, g.nf);
      if (g.N == PP / 2)
        launch(k_z<R, PP, true>, grid, dim3(2 * C::WZ * C::TL), 0, s, ft, g, tb);
      else
        launch(k_z<R, PP, false>, grid, dim3(2 * C::WZ * C::TL), 0, s, ft, g, tb);
    }
  });
}

template <class R>
hipError_t launch_inv_y(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  return dispatch_p(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassIY>;
    dim3 grid(((PP / 2) / C::WS) * g.n, g.nf);
    if (g.N == PP / 2)
      launch(k_inv_y<R, PP, true>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
    else
      launch(k_inv_y<R, PP, false>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
  });
}

template <class R>
hipError_t launch_inv_x(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  // pairs of lines per transform, except for full grids below N = 256 (their
  // carry epilogue) and where x_pairs says no
  bool pairs = g.N >= 256;
  if (!pairs && x_pairs<R>(g.N)) {
    pairs = true;
    for (int k = 0; k < g.nf; ++k) pairs = pairs && ft.f[k].kind != 0 && ft.f[k].kind != 4;
  }
  return dispatch_p(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassIX>;
    const int units = pairs ? g.n * g.n / 2 : g.n * g.n;
    constexpr int UW = C::WC * x_iters<PP, true>();  // units per workgroup
    dim3 grid((units + UW - 1) / UW, g.nf);
    // a launch's grids share the carry rule (the runtime groups by it)
    const bool tri = ft.f[0].tri != 0;
    if (pairs && tri)
      launch(k_inv_x<R, PP, true, true>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
    else if (pairs)
      launch(k_inv_x<R, PP, true, false>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
    else if (tri)
      launch(k_inv_x<R, PP, false, true>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
    else
      launch(k_inv_x<R, PP, false, false>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
  });
}

template <class R>
hipError_t launch_inv_y_fold(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  // g.P is the scaled period S P (>= 4N); the transforms run at P
  if ((g.S != 2 && g.S != 4) || g.P < 4 * g.N || g.P / g.S < 8) return hipErrorInvalidValue;
  return dispatch_p(g.P / g.S, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    // S P <= 1024: doubled grids up to P = 512, quadrupled up to 256
    using C = Cfg<R, PP, kPassIY>;
    if (g.S == 2) {
      dim3 grid((PP / C::WS) * g.N, g.nf);
      launch(k_inv_y_fold<R, PP, 2>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
    } else if constexpr (PP <= 256) {
      dim3 grid((2 * PP / C::WS) * g.N, g.nf);
      launch(k_inv_y_fold<R, PP, 4>, grid, dim3(C::WS * C::TL), 0, s, ft, g, tb);
    }
  });
}

template <class R>
hipError_t launch_inv_x_fold(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  if ((g.S != 2 && g.S != 4) || g.P < 4 * g.N || g.P / g.S < 8) return hipErrorInvalidValue;
  return dispatch_p(g.P / g.S, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassIX>;
    dim3 grid((g.N * g.N / 2 + C::WC - 1) / C::WC, g.nf);
    const bool tri = ft.f[0].tri != 0;
    if (g.S == 2) {
      if (tri) launch(k_inv_x_fold<R, PP, 2, true>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
      else launch(k_inv_x_fold<R, PP, 2, false>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
    } else if constexpr (PP <= 256) {
      // quadrupled grids add no carry
      launch(k_inv_x_fold<R, PP, 4, false>, grid, dim3(C::WC * C::TL), 0, s, ft, g, tb);
    }
  });
}

template <class R>
bool plane_passes_fit(int P) {
  bool ok = false;
  (void)dispatch_p(P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    ok = PP <= kPlaneMaxP && PlaneCfg<R, PP>::LDS <= kPlaneLdsMax;
  });
  return ok;
}

template <class R>
hipError_t launch_fwd_xy(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  return dispatch_p(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using PC = PlaneCfg<R, PP>;
    if constexpr (PP <= kPlaneMaxP && PC::LDS <= kPlaneLdsMax) {
      dim3 grid(g.n, g.nf);
      if (g.N == PP / 2)
        launch(k_fwd_xy<R, PP, true>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
      else
        launch(k_fwd_xy<R, PP, false>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
    }
  });
}

template <class R>
hipError_t launch_inv_yx(const FieldTable& ft, PassGeom g, Tables<R> tb, hipStream_t s) {
  return dispatch_p(g.P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using PC = PlaneCfg<R, PP>;
    if constexpr (PP <= kPlaneMaxP && PC::LDS <= kPlaneLdsMax) {
      dim3 grid(g.n, g.nf);
      const bool tri = ft.f[0].tri != 0;
      if (g.N == PP / 2 && tri)
        launch(k_inv_yx<R, PP, true, true>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
      else if (g.N == PP / 2)
        launch(k_inv_yx<R, PP, true, false>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
      else if (tri)
        launch(k_inv_yx<R, PP, false, true>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
      else
        launch(k_inv_yx<R, PP, false, false>, grid, dim3(PC::NTH), 0, s, ft, g, tb);
    }
  });
}

template <class R>
hipError_t launch_accel(const R* phi, R* g, int N, int L, double h0, hipStream_t s) {
  launch(k_accel<R>, dim3((unsigned)((N * N + 255) / 256), N, L), dim3(256), 0, s, phi, g, N, L, h0);
  return hipGetLastError();
}

template <class R>
hipError_t launch_restrict(const R* fine, const R* fine_rc, R* rc, int N, hipStream_t s) {
  const int n = (N / 2) * (N / 2) * (N / 2);
  launch(k_restrict<R>, dim3((n + 255) / 256), dim3(256), 0, s, fine, fine_rc, rc, N);
  return hipGetLastError();
}

template <class R>
hipError_t launch_pyramid(const PyramidTable& tab, int count, int N, int maxL, hipStream_t s) {
  int blocks = 0;
  for (int k = 1; k < maxL; ++k) {
    const int S = pyramid_cube(N, k), nc = N / S;
    blocks += nc * nc * nc;
  }
  launch(k_pyramid<R>, dim3(blocks, count), dim3(kPyramidThreads), 0, s, tab, N, maxL);
  return hipGetLastError();
}

template <class R>
hipError_t launch_carry_tri(const CarryTable& tab, int count, int N, int n, hipStream_t s) {
  const int NB = N / 2 + 2, per = (NB * NB * NB + 255) / 256;
  if (sizeof(R) == 4 && tab.r[0].comp)
    launch(k_carry_tri<R, true>, dim3(per, count), dim3(256), 0, s, tab, N, n);
  else
    launch(k_carry_tri<R, false>, dim3(per, count), dim3(256), 0, s, tab, N, n);
  return hipGetLastError();
}

template <class R>
hipError_t launch_carry(const CarryTable& tab, int count, int N, int n0, hipStream_t s) {
  const int NB = N / 2 + 2, per = (NB * NB * NB + 255) / 256;
  int nl = 0;
  for (int i = 0; i < count; ++i) nl = std::max(nl, tab.nlev[i]);
  if (nl <= 0) return hipSuccess;
  // a launch is either all compensated or all plain (runtime groups them)
  if (sizeof(R) == 4 && tab.r[0].comp)
    launch(k_carry<R, true>, dim3(per * nl, count), dim3(256), 0, s, tab, N, n0);
  else
    launch(k_carry<R, false>, dim3(per * nl, count), dim3(256), 0, s, tab, N, n0);
  return hipGetLastError();
}

hipError_t launch_green(int P, double beta, const double2* tw, double* t1, double* t2, double* out,
                        hipStream_t s) {
  return dispatch_p<1024>(P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<double, PP, kPassOther>;
    constexpr int H = PP / 2 + 1;
    dim3 grid((H * H + C::WC - 1) / C::WC);
    dim3 block(C::WC * C::TL);
    launch(k_green<PP>, grid, block, 0, s, 0, beta, tw, (const double*)nullptr, t1);
    launch(k_green<PP>, grid, block, 0, s, 1, beta, tw, (const double*)t1, t2);
    launch(k_green<PP>, grid, block, 0, s, 2, beta, tw, (const double*)t2, out);
  });
}

template <class R>
size_t green_layout_elems(int P) {
  size_t n = 0;
  (void)dispatch_p<1024>(P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    n = (size_t)(PP / 2 + 1) * (PP / 2 + 1) * (PP / 2);
  });
  return n;
}

template <class R>
hipError_t launch_green_layout(int P, const double* octant, R* gz, R* gn, hipStream_t s) {
  return dispatch_p<1024>(P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    const size_t n = (size_t)(PP / 2 + 1) * (PP / 2 + 1) * (PP / 2);
    launch(k_green_layout<R, PP>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, octant,
                       gz, gn);
  });
}

hipError_t launch_round_f32(const double* in, float* out, size_t n, hipStream_t s) {
  launch(k_round_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

template <class R>
hipError_t launch_fft_lines(const void* in, void* out, int P, int nlines, int dir, const void* tw,
                            hipStream_t s) {
  using T = cplx<R>;
  return dispatch_p(P, [&](auto pc) {
    constexpr int PP = decltype(pc)::value;
    using C = Cfg<R, PP, kPassOther>;
    dim3 grid((nlines + C::WC - 1) / C::WC), block(C::WC * C::TL);
    if (dir < 0)
      launch(k_fft_lines<R, PP, -1>, grid, block, 0, s, (const T*)in, (T*)out,
                         nlines, (const T*)tw);
    else
      launch(k_fft_lines<R, PP, +1>, grid, block, 0, s, (const T*)in, (T*)out,
                         nlines, (const T*)tw);
  });
}

#define NMC_INSTANTIATE(R)                                                                        \
  template hipError_t launch_fwd_x<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);       \
  template hipError_t launch_fwd_y<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);       \
  template hipError_t launch_z<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);           \
  template hipError_t launch_inv_y<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);       \
  template hipError_t launch_inv_x<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);       \
  template hipError_t launch_inv_y_fold<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);  \
  template hipError_t launch_inv_x_fold<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);  \
  template hipError_t launch_fwd_xy<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);      \
  template hipError_t launch_inv_yx<R>(const FieldTable&, PassGeom, Tables<R>, hipStream_t);      \
  template bool plane_passes_fit<R>(int);                                                         \
  template hipError_t launch_restrict<R>(const R*, const R*, R*, int, hipStream_t);               \
  template hipError_t launch_pyramid<R>(const PyramidTable&, int, int, int, hipStream_t);          \
  template hipError_t launch_carry<R>(const CarryTable&, int, int, int, hipStream_t);              \
  template hipError_t launch_carry_tri<R>(const CarryTable&, int, int, int, hipStream_t);          \
  template hipError_t launch_accel<R>(const R*, R*, int, int, double, hipStream_t);                \
  template hipError_t launch_fft_lines<R>(const void*, void*, int, int, int, const void*, hipStream_t); \
  template hipError_t launch_green_layout<R>(int, const double*, R*, R*, hipStream_t);                 \
  template size_t green_layout_elems<R>(int);

NMC_INSTANTIATE(double)
NMC_INSTANTIATE(float)

}  // namespace nmc
