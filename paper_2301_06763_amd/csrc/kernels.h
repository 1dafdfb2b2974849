// Host-side launch interface of the nested-mesh convolution kernels.
// Every launcher enqueues asynchronously on `stream` and returns the launch
// status; shapes are validated by the caller (runtime.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

namespace nmc {

// One grid to convolve (Sect. 3 of the paper) on the doubled period P.  Its
// input occupies cells [0, nin) per axis and its output rows [olo, olo + nout):
//  * kind 0, a full level Omega^m: nin = nout = N, olo = 0; density rho with
//    the child region replaced by its restriction rc when rc is set;
//  * kind 1, the child region of a level alone, embedded with a one-cell
//    margin in a box of nin = nout = N/2 + 2 cells per axis (the stencil box
//    [N/4 - 1, 3N/4] of the level): density rc (or rho's child region when
//    rc is null), zero in the margin.  Its potential C on the box gives the
//    hole potential of Sect. 4 by linearity: Phi_hole = Phi - C;
//  * kind 2, the level with its child region zeroed (Omega^m_hole of Sect. 4,
//    Fig. 5): nin = N, output only on the stencil box (olo = N/4 - 1,
//    nout = N/2 + 2);
//  * kind 3 (modified method, Sect. 7 and Appendix B), the doubled grid of
//    the pair (l, l+1): level l+1's density (rho, rc) on a grid of 2N cells
//    of level l+1's spacing spanning level l, period 2P: its N input rows
//    sit at frame rows [N/2, 3N/2), its output rows are [0, 2N), reduced to
//    level l's N cells per axis by the inverse passes (out: level l's
//    potential, to which the reduced values and the carry S are added);
//  * kind 4 (modified method), kind 2's grid with full output: out gets the
//    hole potential on all N^3 cells and Sout its stencil box;
//  * kind 5 (three-level scheme of Appendix B), kind 3 with the input's
//    child region zeroed (the doubled hole grid).  Kinds 3 and 5 also serve
//    at scale 4 (quadrupled grid: 4N cells of level l+2's spacing, period
//    4P, input rows at [3N/2, 5N/2)); PassGeom.S gives the scale.
struct FieldDesc {
  const void* rho;   // level density [N][N][N] (x fastest), caller-owned
  const void* rc;    // restriction data of the child region (pyramid slab of level l+1), or null
  void* A;           // workspace [nin][nin][P/2] complex: x-pass output, y-inverse output
  void* B;           // workspace [nin][P][P/2] complex, z rows zrow_pitch apart: y-pass output, z-pass in place
  void* out;         // kind 0: potential [N][N][N]; kinds 1, 2: box [(N/2+2)^3]
  const void* S;     // kind 0, level >= 1: carried coarse potential S_{l-1} on the box (hi)
  const void* Slo;   // its compensation term (FP32 path) or null
  void* Sout;        // kind 0 with kind-1 boxes, level < L-1: S_l = Phi(Omega^l) - C_l (hi)
  void* Slo_out;     // its compensation term (FP32 path) or null
  const void* C;     // with Sout: C_l on the box
  double scale;      // -G h^2 / P^3 (mass = rho h^3, kernel 1/(h |d|), 1/P^3 of the inverse)
  long long rslab;   // elements between the restriction slabs of consecutive levels
  int rdepth;        // terms of the restricted value (1: rc holds the finished restriction)
  int kind;          // 0 full level, 1 child-region box, 2 level with its child region zeroed,
                     // 3 doubled grid, 4 hole grid with full output
  int comp;          // FP32: compensated (two-term) carry
  int tri;           // carry by the tensor-product rule (NMC_PROLONG_TRILINEAR), else Eqs. 3-6
};

// Elements between consecutive z rows of a grid's B (a z row holds P rows ky
// of P/2 complex values of cbytes bytes each).  The z pass reads and writes
// B down its columns, one value per z row; at a power-of-two row pitch (2 MB
// at P = 512 in FP64) the values of a column, and those that neighbouring
// workgroups touch at the same time, fall on the same few HBM channels.  A
// plain read and write of 128-byte column runs of such a B moves 4.2 TB/s
// at the power-of-two pitch and 4.5 TB/s (4.9 TB/s with the rows ky
// fastest across workgroups) with 256 bytes more per z row.
#ifndef NMC_ZROW_PAD
#define NMC_ZROW_PAD 256
#endif
__host__ __device__ constexpr size_t zrow_pitch(int P, size_t cbytes) {
  return (size_t)P * (P / 2) + (size_t)NMC_ZROW_PAD / cbytes;
}

// Restriction data (Sect. 2: the density of a level's child region is the
// mean over the 2x2x2 children of the next finer level, whose own child
// region is restricted in turn).  Unrolled, the restricted value of cell c
// of level l's child region is a sum over the finer levels k > l of the
// mean of m_k over c's footprint on level k, where m_k is level k's density
// with its own child region zeroed (k < L-1).  When N is a multiple of 2^L
// every footprint is an aligned block of 2^(k-l) cells per axis, so with
// block means of m_k at every size 2^d stored per level ("pyramid"), the
// restricted value is L-1-l loads.  Level k's slab holds, for d = 1, 2, ...,
// the block means at size 2^d ((N >> d)^3 values each, x fastest), one after
// the other; the slab of level k starts (k-1)*slab elements after level 1's.
// rdepth = 1 reads a single finished value per cell (cascaded restriction).
inline long long pyramid_slab(int N, int L) {
  long long s = 0;
  for (int d = 1; d <= L - 1 && (N >> d) > 0; ++d) s += (long long)(N >> d) * (N >> d) * (N >> d);
  return s;
}
inline bool pyramid_exact(int N, int L) { return L >= 2 && L - 1 <= 5 && N % (1 << L) == 0; }
constexpr int kMaxPyramidDepth = 5;  // blocks up to 32^3 cells per workgroup
// Edge of the cube of level k a workgroup reduces: a multiple of 2^k that
// divides N, grown up to 16 cells when N allows.
__host__ __device__ inline int pyramid_cube(int N, int k) {
  int S = 1 << k;
  while (S < 16 && N % (2 * S) == 0) S *= 2;
  return S;
}

struct PyramidDesc {
  const void* rho;  // the request's densities, L levels of N^3
  void* pyr;        // slab of level 1; level k at (k-1)*slab
  long long slab;
  int L;
};
constexpr int kMaxPyramidsPerLaunch = 24;
struct PyramidTable {
  PyramidDesc r[kMaxPyramidsPerLaunch];
};

// Carry cascade of the hole pipeline (Sect. 4, Eqs. 3-6), on the stencil box
// [N/4-1, 3N/4]^3 of every level (NB = N/2+2 cells per axis, x fastest):
// S_0 = Phi^0_hole, S_n = Prolong(S_{n-1}) + Phi^n_hole.
struct CarryDesc {
  const void* hole;    // Phi^n_hole of level n at hole + n * box
  void* S;             // S_n (hi) at S + n * 2 * box, its compensation term box elements later
  long long box;       // elements per box (padded)
  int comp;            // FP32: keep the two-term (hi, lo) sums
};
constexpr int kMaxCarriesPerLaunch = 24;
struct CarryTable {
  CarryDesc r[kMaxCarriesPerLaunch];
  int nlev[kMaxCarriesPerLaunch];  // levels n0..n0+nlev-1 of this launch, per request
};
constexpr int kMaxCarryDepth = 4;  // levels per launch: each S_n from S_{n0-1} in one recursion

constexpr int kMaxFieldsPerLaunch = 24;
struct FieldTable {
  FieldDesc f[kMaxFieldsPerLaunch];
};

struct PassGeom {
  int N;     // cells per axis of the level
  int P;     // padded period (power of two >= 2N; S times the level's for scaled grids)
  int n;     // largest nin (x, y passes) or nout (inverse passes) of the launch's grids
  int nf;    // grids in this launch
  int S;     // scale factor of the launch's grids: 1, or 2 (doubled) / 4 (quadrupled) for kinds 3, 5
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

// Timing of the next kernel launch (profiling): when set, the next kernel a
// launcher below enqueues records `start` as it begins and `stop` as it ends
// (hipExtLaunchKernel), and the pair is cleared.  Per host thread.
// take_next_launch_events clears a pair nothing consumed and says whether
// there was one.
void set_next_launch_events(hipEvent_t start, hipEvent_t stop);
bool take_next_launch_events();

// Forward passes and the fused z pass.
template <class R> hipError_t launch_fwd_x(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_fwd_y(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_z(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
// Inverse passes (output-pruned).
template <class R> hipError_t launch_inv_y(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_inv_x(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
// Inverse passes of the scaled grids (kinds 3, 5: modified method) after
// their z pass, with the S^3 mean taken in the spectrum (each transform at
// the level's period g.P / g.S): I2 (sum of z rows S j .. S j + S - 1, y
// fold, rows y < N kept) and I1 (x fold, C2R, the mean added to out, plus
// the carry S when set).  g.N is the level's N, g.P the scaled period
// (>= 4N), g.S = 2 or 4; tb its tables.
template <class R> hipError_t launch_inv_y_fold(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_inv_x_fold(const FieldTable&, PassGeom, Tables<R>, hipStream_t);

// Fused plane passes for P <= 64 when a plane fits the LDS
// (plane_passes_fit): X+Y in one launch, I2+I1 in one launch; the A
// workspace is not used.  g.n is the largest nin (fwd_xy) or nout (inv_yx).
template <class R> bool plane_passes_fit(int P);
template <class R> hipError_t launch_fwd_xy(const FieldTable&, PassGeom, Tables<R>, hipStream_t);
template <class R> hipError_t launch_inv_yx(const FieldTable&, PassGeom, Tables<R>, hipStream_t);

// Restriction of level l+1 onto the child region of level l, one level per
// launch (any N); fine_rc is the finished restriction of level l+1 or null.
template <class R>
hipError_t launch_restrict(const R* fine, const R* fine_rc, R* rc_out, int N, hipStream_t);
// Block-mean pyramids of every level k >= 1 of up to kMaxPyramidsPerLaunch
// requests in one launch (requires pyramid_exact(N, L) for each).
template <class R>
hipError_t launch_pyramid(const PyramidTable&, int count, int N, int maxL, hipStream_t);
// S_n for n = n0 .. n0 + nlev - 1 (nlev <= kMaxCarryDepth), each from S_{n0-1}
// (S_0 = Phi^0_hole when n0 = 1) by unrolling the cascade, in one launch.
// Every request of the table has the same comp.
template <class R>
hipError_t launch_carry(const CarryTable&, int count, int N, int n0, hipStream_t);
// S_n for level n alone (1 <= n <= nlev per request) by the tensor-product
// rule (NMC_PROLONG_TRILINEAR), from S_{n-1} (S_0 = Phi^0_hole).
template <class R>
hipError_t launch_carry_tri(const CarryTable&, int count, int N, int n, hipStream_t);

// Gravitational acceleration of a solved nested potential phi [L][N][N][N]
// into g [L][3][N][N][N] (six-point stencil, Appendix A methods A and B).
template <class R>
hipError_t launch_accel(const R* phi, R* g, int N, int L, double h0, hipStream_t);

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
