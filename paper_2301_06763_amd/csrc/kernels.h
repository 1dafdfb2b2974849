// Host-side launch interface of the nested-mesh convolution kernels.
// Every launcher enqueues asynchronously on `stream` and returns the launch
// status; shapes are validated by the caller (runtime.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

namespace nmc {

// One grid to convolve: a full level (Omega^m) or a level with its cavity
// zeroed (Omega^m_hole), Sect. 4 of the paper.
struct FieldDesc {
  const void* rho;   // level density [N][N][N] (x fastest), caller-owned
  const void* rc;    // restricted density of the child region [(N/2)^3], or null
  void* A;           // workspace [N][N][P/2] complex: x-pass output, y-inverse output
  void* B;           // workspace [N][P][P/2] complex: y-pass output, z-pass in place
  void* out;         // full: potential [N][N][N]; hole: stencil box [(N/2+2)^3]
  const void* S;     // full, level >= 1: carried coarse potential (hi) on the stencil box
  const void* Slo;   // its compensation term (FP32 path) or null
  double scale;      // -G h^2 / P^3 (mass = rho h^3, kernel 1/(h |d|), 1/P^3 of the inverse)
  int hole;          // 1 for Omega_hole
  int has_carry;     // full field of a level >= 1
};

constexpr int kMaxFieldsPerLaunch = 24;
struct FieldTable {
  FieldDesc f[kMaxFieldsPerLaunch];
};

struct PassGeom {
  int N;     // cells per axis
  int P;     // padded period (power of two >= 2N)
  int nf;    // fields in this launch
  int flags;
};

template <class R>
struct Tables {
  const typename std::conditional<sizeof(R) == 8, double2, float2>::type* tw;  // exp(-2 pi i j/P), j < P
  // Real Green spectrum in the z pass's reading order: gz[kyp][tile][kzp][w]
  // for kx = tile*W + w < P/2 (W = the z pass's tile width) and gn[kyp][kzp]
  // for kx = P/2; kyp, kzp in [0, P/2] (the spectrum is even in ky and kz).
  const R* gz;
  const R* gn;
};

// Forward passes and the fused z pass.
template <class R> hipError_t launch_fwd_x(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_fwd_y(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_z(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
// Inverse passes (output-pruned).
template <class R> hipError_t launch_inv_y(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_inv_x(const FieldTable&, PassGeom, Tables<R>, hipStream_t);

// Restriction of level l+1 onto the child region of level l.
template <class R>
hipError_t launch_restrict(const R* fine, const R* fine_rc, R* rc_out, int N, hipStream_t);
// S_n = Prolong(S_{n-1}) + Phi^n_hole on the stencil box (hi/lo pair; lo may be null).
template <class R>
hipError_t launch_carry(const R* s_hi, const R* s_lo, const R* hole, R* o_hi, R* o_lo, int N,
                        int compensated, hipStream_t);

// Green spectrum, FP64: three separable passes over the even octant.
hipError_t launch_green(int P, double beta, const double2* tw, double* t1, double* t2, double* out,
                        hipStream_t);
hipError_t launch_round_f32(const double* in, float* out, size_t n, hipStream_t);
// Reorder the FP64 octant [kz][ky][kx] into the z pass's layout (gz, gn) for R.
template <class R>
hipError_t launch_green_layout(int P, const double* octant, R* gz, R* gn, hipStream_t);
template <class R>
size_t green_layout_elems(int P);  // elements of gz (gn has (P/2+1)^2)

// Batched 1-D complex FFT of contiguous lines (diagnostic entry point).
template <class R>
hipError_t launch_fft_lines(const void* in, void* out, int P, int nlines, int dir, const void* tw,
                            hipStream_t);

}  // namespace nmc
