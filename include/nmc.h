/*
 * nmc.h - C ABI of libnmc, the MI355X (gfx950) implementation of the
 * convolution method for the gravitational potential on nested Cartesian
 * meshes (Vorobyov, McKevitt, Kulikov, Elbakyan, A&A 2023, arXiv:2301.06763).
 *
 * Problem (Sect. 2 and 4 of the paper): given densities rho on L concentric
 * nested grids Omega^1 > ... > Omega^L of N^3 cells each, level m+1 covering
 * the central half (per axis) of level m with half the cell size, find the
 * potential Phi(Omega^m) on every level.
 *
 * Method: on every level (Sect. 3) the potential of the cell masses M = rho h^3
 * is the discrete sum Phi = -G sum M / |r - r'| (Eq. 10) with the self-cell
 * term of Eq. 13, evaluated as a zero-padded FFT convolution on a doubled
 * periodic mesh (Fig. 4).  The nested mesh is split into full grids Omega^m
 * and grids with a zeroed cavity Omega^m_hole (Sect. 4, Fig. 5); the result
 * on Omega^n is Phi^n plus the hole potentials of all coarser grids
 * interpolated onto it (Eq. 14).
 *
 * Conventions for every array argument:
 *   - Densities and potentials: [L][N][N][N], level 0 = coarsest, index order
 *     [z][y][x] with x fastest, contiguous, element type double (NMC_F64) or
 *     float (NMC_F32).  Level l has cell size h0 / 2^l and is centred on the
 *     origin; level l+1 covers cells [N/4, 3N/4) of level l on each axis.
 *   - Pointers named "device" must be HIP device memory of the context's
 *     device; the caller allocates and frees them.
 *   - Every call returns NMC_OK (0) or a negative status.  All argument
 *     validation happens before any device work is enqueued; on an error no
 *     caller buffer is written.  nmc_last_error() describes the last failure.
 *   - Work is enqueued asynchronously on the caller's hipStream_t (passed as
 *     void*; NULL = the null stream).  Results are valid after the stream is
 *     synchronised.  Device faults surface at a later call or the sync.
 *   - A context is not thread-safe: use one per host thread.
 */
#ifndef NMC_H
#define NMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmc_ctx nmc_ctx;

typedef enum { NMC_F64 = 0, NMC_F32 = 1 } nmc_precision;

enum {
  NMC_OK = 0,
  NMC_EINVAL = -1,       /* invalid argument (null pointer, bad N/L/h0/G/refine, aliasing) */
  NMC_ENOMEM = -2,       /* footprint above the context's HBM budget, or allocation failure */
  NMC_EDEVICE = -3,      /* HIP runtime error (text in nmc_last_error) */
  NMC_EUNSUPPORTED = -4, /* N beyond the supported range (padded period above 512) */
  NMC_EAGAIN = -5        /* serving: ticket not finished yet / nothing admitted yet */
};

/* Flag bits for nmc_solve / nmc_request.flags. */
enum {
  /* Keep the caller's coarse density under finer grids.  Default: replace it
   * by the mean of the 2^3 finer cells below, cascaded from the finest level
   * (mass conserving; the paper leaves the coarse mass under a finer grid
   * unspecified). */
  NMC_NO_RESTRICT = 1u << 0,
  /* Carry the coarser levels' hole potentials to finer cells with the
   * tensor-product rule (weights 3/4 and 1/4 per axis over the 8
   * surrounding coarse cells) instead of the default: Eqs. 3-6 applied to
   * every fine cell (3/4 of the parent plus 1/4 of the diagonal neighbour).
   * Both are exact on linear fields (Sect. 4 leaves the interpolation
   * open). */
  NMC_PROLONG_TRILINEAR = 1u << 1,
  /* FP32 only: plain FP32 cross-level sums instead of the compensated
   * (two-term) carry.  For ablation. */
  NMC_F32_UNCOMPENSATED = 1u << 2,
  /* nmc_solve only: always launch the kernels directly.  Default: the second
   * and later calls with identical arguments (same pointers, shape, h0, G,
   * precision and flags) replay a captured HIP graph that owns its own
   * workspace, which removes the per-kernel launch cost. */
  NMC_NO_GRAPH = 1u << 3,
  /* Enqueue every grid on hip_stream only.  Default from N = 128 (where the
   * hole potentials come from child-region boxes): the boxes run on a second,
   * library-owned stream forked from and joined back into hip_stream,
   * overlapping the full grids' passes. */
  NMC_ONE_STREAM = 1u << 4,
  /* Use the separate X, Y, I2 and I1 passes even where fused plane passes
   * apply (P <= 64, hole-grid formulation; default there: one XY and one
   * I2+I1 launch per kind of grid, each z plane kept in LDS).  For
   * ablation.  In a batch, ONE_STREAM and NO_FUSED_PLANES are taken from the
   * first request of each group of equal N, precision and method. */
  NMC_NO_FUSED_PLANES = 1u << 5,
  /* The modified convolution method of Sect. 7 and Appendix B (Eqs. B.1,
   * B.2), which keeps the dipole moments between neighbouring levels: for
   * every level l < L-1, phi[l] = Phi^l_hole + the potential of level l+1's
   * masses convolved on the doubled grid (2N cells of level l+1's spacing
   * spanning level l, period 2P) and averaged over the 2^3 doubled cells of
   * each level-l cell + the coarser hole potentials carried down as in
   * Eq. 14; the finest level is unchanged.  Needs 2P <= 1024 (every N up to
   * 256) and a larger workspace (nmc_footprint_bytes_flags). */
  NMC_MODIFIED = 1u << 6,
  /* The modified method with Appendix B's scheme for dipoles across three
   * neighbouring grids (implies NMC_MODIFIED): every level l with two finer
   * levels takes Phi^l_hole + level l+1's density with its child region
   * zeroed on the doubled grid + level l+2's density on a quadrupled grid
   * (4N cells of level l+2's spacing spanning level l, period 4P, averaged
   * over the 4^3 cells of each level-l cell) + the carry; the two finest
   * levels as with NMC_MODIFIED.  Needs 4P <= 1024 (N <= 128) when L >= 3. */
  NMC_MODIFIED3 = 1u << 7
};

/* Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * library's workspace and its cached Green-spectrum tables together (0 = no
 * cap; the short-lived buffers of a table's first build are not counted).
 * Over the budget the context releases cached workspace blocks and then the
 * least recently used tables of periods the current work does not need
 * (after synchronising the device; captured graph replays are dropped with
 * them and recaptured on demand).  *out receives the context.  Errors:
 * NMC_EINVAL (out null, bad device), NMC_EDEVICE. */
int nmc_create(nmc_ctx** out, int hip_device, size_t hbm_budget_bytes);

/* Destroy a context after synchronising its device work; frees every
 * library-owned buffer.  Caller buffers are untouched.  NULL is a no-op. */
void nmc_destroy(nmc_ctx* ctx);

/* Text of the last failure on this context (static storage owned by the
 * context; valid until the next call on it).  Never NULL. */
const char* nmc_last_error(const nmc_ctx* ctx);

/* Device workspace (bytes) one solve of this shape needs: the per-grid FFT
 * buffers of all 2L-1 grids plus the restriction and carry buffers.  Pure
 * host arithmetic.  Errors: NMC_EINVAL, NMC_EUNSUPPORTED. */
int nmc_footprint_bytes(int N, int L, nmc_precision p, size_t* bytes);

/* The same for a solve with these flags (NMC_MODIFIED adds the doubled
 * grids' FFT buffers, NMC_MODIFIED3 also the quadrupled grids').  Errors:
 * NMC_EINVAL, NMC_EUNSUPPORTED (also for NMC_MODIFIED3 with N above 128
 * and L >= 3). */
int nmc_footprint_bytes_flags(int N, int L, nmc_precision p, unsigned flags, size_t* bytes);

/* Solve one nested mesh (Sect. 4, Eq. 14).
 *   rho   device, [L][N][N][N] densities (read only, never written)
 *   phi   device, [L][N][N][N] output; phi[l] = Phi(Omega^(l+1)) on all N^3
 *         cells of level l, including cells covered by finer levels.
 *         Must not overlap rho.
 *   N     cells per axis, multiple of 4, 4 <= N <= 256
 *   L     levels, 1 <= L <= 16
 *   h0    coarsest cell size (> 0, finite)
 *   refine  refinement factor between levels; must be 2
 *   G     gravitational constant (finite)
 *   p     element type of rho and phi and arithmetic of the FFT path
 *   flags NMC_NO_RESTRICT, NMC_PROLONG_TRILINEAR, NMC_F32_UNCOMPENSATED, NMC_NO_GRAPH, NMC_ONE_STREAM,
 *         NMC_NO_FUSED_PLANES, NMC_MODIFIED, NMC_MODIFIED3
 *   hip_stream  hipStream_t to enqueue on.  The hole grids and the carry
 *         cascade run on a second, library-owned stream that is forked from
 *         and joined back into hip_stream, so completion is ordered on
 *         hip_stream alone.
 * Errors: NMC_EINVAL, NMC_EUNSUPPORTED, NMC_ENOMEM, NMC_EDEVICE. */
int nmc_solve(nmc_ctx* ctx, const void* rho, void* phi, int N, int L, double h0, int refine,
              double G, nmc_precision p, unsigned flags, void* hip_stream);

/* Largest workspace nmc_solve_noalloc serves (64 MiB): e.g. N = 32 at any L
 * in FP64 and FP32, N = 64 up to L = 3 (FP64) or L = 5 (FP32). */
#define NMC_SCRATCH_BYTES ((size_t)64 << 20)

/* nmc_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, semantics and results as nmc_solve (the same kernels; every grid
 * on hip_stream, never a graph replay), but it calls no hipMalloc, hipFree or
 * other allocating routine.
 *   Workspace: a static array of NMC_SCRATCH_BYTES in the library's device
 *   code, one per GPU (held until the process ends; its address is looked up
 *   once per device by nmc_create).  Every call on one GPU uses the same
 *   array and leaves its contents behind: calls whose work overlaps on one
 *   GPU (other streams, other contexts, other host threads) race and must be
 *   ordered by the caller.  Nothing in it needs clearing between calls.
 *   Tables: the Green tables of every period the solve needs (P, and 2P / 4P
 *   with NMC_MODIFIED / NMC_MODIFIED3) must already be resident in ctx, built
 *   by an earlier nmc_solve of the same N and method or by nmc_green_spectrum
 *   of that N (and 2N, 4N); a table evicted under the context's budget must be
 *   rebuilt the same way.
 * Errors: as nmc_solve; NMC_ENOMEM when the workspace
 * (nmc_footprint_bytes_flags) exceeds NMC_SCRATCH_BYTES or a table is not
 * resident (nothing is enqueued then). */
int nmc_solve_noalloc(nmc_ctx* ctx, const void* rho, void* phi, int N, int L, double h0, int refine,
                      double G, nmc_precision p, unsigned flags, void* hip_stream);

/* One request of a batch (same meaning as the nmc_solve arguments; the
 * refinement factor is 2). */
typedef struct {
  const void* rho;
  void* phi;
  int N;
  int L;
  double h0;
  double G;
  nmc_precision p;
  unsigned flags;
} nmc_request;

/* Solve `count` independent nested meshes (Sect. 4: the grids of a solve are
 * independent, and so are solves).  Requests of equal N, precision and
 * method (original, NMC_MODIFIED, NMC_MODIFIED3; and carry rule) share
 * every FFT pass launch.  Each result is bitwise identical to the same request solved
 * alone.  All requests are validated before any work. */
int nmc_solve_batch(nmc_ctx* ctx, const nmc_request* reqs, int count, void* hip_stream);

/* ---- Serving: continuous batching over library-owned streams ----------
 * Requests are queued by nmc_serve_submit.  Every nmc_serve_tick retires
 * finished batches (returning their workspace), then admits queued requests
 * in arrival order while the summed nmc_footprint_bytes of in-flight work
 * stays within the budget, groups the admitted ones as nmc_solve_batch does
 * (N, precision, method and carry rule) and launches each group as one
 * batched solve on the next serving stream, so new work overlaps the work
 * already on the device.  Under a budget the batches' workspace comes from
 * one device allocation made at the first serving launch (what the budget
 * leaves beside the Green tables, the workspace of solves in flight and a
 * sixteenth of the budget, at most 1 GiB, kept for tables of other periods)
 * and used as a ring, so a serving loop at its budget makes no allocation,
 * free or device-wide wait; a batch that does not fit beside the batches in
 * flight waits for the next tick, and one larger than the whole ring (with
 * nothing in flight) releases it and runs on workspace of its own, as a
 * solve does.  The allocation is released when a solve outside the serving
 * loop needs its room and no batch is in flight.
 * rho/phi of a submitted request must stay valid until it is reported
 * done. */

/* Queue a request; *ticket receives its id.  hip_stream is the stream on
 * which the caller wrote req->rho (and last used req->phi): an event is
 * recorded on it here, and the batch that solves the request waits for that
 * event on its serving stream, so work the caller enqueued on hip_stream
 * before this call is ordered before the solve.  The result is complete (and
 * may be read from any stream) once nmc_serve_poll reports it done or
 * nmc_serve_take_completed returns its ticket.  NMC_ENOMEM if the request
 * alone exceeds the budget (it could never be admitted); NMC_EINVAL /
 * NMC_EUNSUPPORTED as for nmc_solve; NMC_EDEVICE if the event cannot be
 * recorded. */
int nmc_serve_submit(nmc_ctx* ctx, const nmc_request* req, void* hip_stream, uint64_t* ticket);

/* One scheduler step (non-blocking).  *launched (may be NULL) receives the
 * number of requests launched in this step.  On an error return every request
 * that was not launched stays queued, in arrival order: NMC_ENOMEM when a
 * batch does not fit the budget with nothing in flight, NMC_EDEVICE when a
 * launch failed (message in nmc_last_error). */
int nmc_serve_tick(nmc_ctx* ctx, int* launched);

/* *done = 1 once the ticket's result is complete on the device (the
 * scheduler is ticked first).  NMC_EINVAL for an unknown ticket. */
int nmc_serve_poll(nmc_ctx* ctx, uint64_t ticket, int* done);

/* Move up to `cap` tickets that completed since the previous call into
 * out[0..*n-1] (oldest first); the scheduler is ticked first.  The tickets are
 * then forgotten by the context (later polls of them return NMC_EINVAL). */
int nmc_serve_take_completed(nmc_ctx* ctx, uint64_t* out, int cap, int* n);

typedef struct {
  uint64_t submitted, admitted, completed, batches;
  uint64_t queued;          /* waiting for admission */
  uint64_t inflight;        /* launched, not yet retired */
  size_t inflight_bytes;    /* workspace held by in-flight batches */
  size_t budget_bytes;      /* admission budget (0 = unlimited) */
  size_t peak_inflight_bytes;
  size_t green_cache_bytes; /* Green-spectrum tables held by the context */
  size_t arena_bytes;       /* serving workspace allocation held (budget set; 0 when released) */
} nmc_serve_stats;

int nmc_serve_stats_get(nmc_ctx* ctx, nmc_serve_stats* out);

/* Block until every submitted request is complete. */
int nmc_serve_drain(nmc_ctx* ctx);

/* ---- Gravitational acceleration ------------------------------------------
 * g = -grad Phi on every level of a nested-mesh potential (Sect. 2: the
 * six-point central stencil, g_x = -(Phi[i+1] - Phi[i-1]) / (2 dx_m)), with
 * the rules of Appendix A next to the coarse-fine interfaces: at a level's
 * outermost cells (levels >= 2 in the paper's numbering) the missing
 * neighbour is the boundary value interpolated from the next coarser level
 * by Eqs. 3-6 (method A); at a coarse cell next to the finer grid, a
 * neighbour inside the child region takes the arithmetic mean of the finer
 * level's potential over the 2^3 cells it covers (method B).  The coarsest
 * level's outer faces use the second-order one-sided difference; cells
 * covered by a finer level use their own level's values.
 *   phi: device, [L][N][N][N], x fastest, element type p (as written by
 *        nmc_solve); read only.
 *   g:   device, [L][3][N][N][N] (components x, y, z, each x fastest),
 *        element type p; caller-owned; must not overlap phi.
 *   N, L, h0: as for nmc_solve (h0 = coarsest cell width).
 * Enqueued asynchronously on hip_stream; no workspace.  Errors: NMC_EINVAL
 * (null or overlapping pointers, N % 4 != 0 or N < 4, L outside [1, 16],
 * h0 not positive and finite, unknown precision), NMC_EUNSUPPORTED (N above
 * 256), NMC_EDEVICE (launch failure). */
int nmc_acceleration(nmc_ctx* ctx, const void* phi, void* g, int N, int L, double h0,
                     nmc_precision p, void* hip_stream);

/* ---- Diagnostics (same kernels as the solve path) --------------------- */

/* Copy the cached real Green spectrum of period P = nmc_period(N) into
 * `out` (device, (P/2+1)^3 elements of type p, index [kz][ky][kx]), building
 * it first if needed.  It is the unnormalised DFT over the doubled periodic
 * mesh of the inverse cell-centre distance (cell units), with the self-cell
 * integral of Eq. 13 at offset 0 (Sect. 3, Fig. 4). */
int nmc_green_spectrum(nmc_ctx* ctx, int N, nmc_precision p, void* out, void* hip_stream);

/* Padded period used for N: the smallest power of two >= 2N (Sect. 3 doubles
 * the mesh; any period >= 2N-1 gives the same linear convolution).  Returns
 * 0 for unsupported N. */
int nmc_period(int N);

/* Batched unnormalised 1-D complex FFT of `nlines` contiguous lines of P
 * points (interleaved re/im, element type p) with the solve path's FFT
 * stages; dir = -1 forward (exp(-2 pi i jk/P)), +1 inverse.  in/out device,
 * may alias.  P in {8, ..., 512}. */
int nmc_fft_lines(nmc_ctx* ctx, const void* in, void* out, int P, int nlines, int dir,
                  nmc_precision p, void* hip_stream);

/* ---- Per-pass profiling --------------------------------------------------
 * When enabled, every pass launch of nmc_solve / nmc_solve_batch / serving is
 * bracketed by two HIP events recorded on the stream it is launched on, and
 * the pass's algorithmic HBM bytes (the bytes the pruned method must read and
 * write for the grids of that launch) are accumulated.  Reading synchronises
 * on the recorded events. */
enum {
  NMC_PASS_RESTRICT = 0, NMC_PASS_X = 1, NMC_PASS_Y = 2, NMC_PASS_Z = 3, NMC_PASS_IY = 4,
  NMC_PASS_IX_SECOND = 5, /* last pass of the hole grids or child-region boxes */
  NMC_PASS_CARRY = 6,     /* carry cascade (hole-grid formulation only) */
  NMC_PASS_IX_FULL = 7,
  /* fused plane passes (P <= 64, used in place of X+Y and I2+I1): */
  NMC_PASS_XY = 8, NMC_PASS_IYX_SECOND = 9, NMC_PASS_IYX_FULL = 10,
  NMC_PASS_ACCEL = 11,    /* nmc_acceleration */
  NMC_PASS_IX_DOUBLED = 12, /* NMC_MODIFIED(3): last pass of the doubled / quadrupled grids (means, sums) */
  NMC_NUM_PASSES = 13
};

typedef struct {
  uint64_t launches;  /* kernel launches recorded */
  double total_ms;    /* summed event-to-event time of those launches */
  double bytes;       /* summed algorithmic bytes of those launches */
} nmc_pass_stat;

/* on = 1 enables recording (and clears earlier records), 0 disables. */
int nmc_profile_enable(nmc_ctx* ctx, int on);

/* Fill out[0..NMC_NUM_PASSES-1] with the totals since the last enable or
 * read, then clear them.  Blocks until the recorded events complete. */
int nmc_profile_read(nmc_ctx* ctx, nmc_pass_stat* out);

/* Name of a pass id ("x", "z", ...), or "?" */
const char* nmc_pass_name(int pass);

#ifdef __cplusplus
}
#endif

#endif /* NMC_H */
