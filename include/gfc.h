/*
 * gfc.h - C ABI of the MI355X (gfx950) Green Function Convolution solver.
 *
 * The solver turns a gradient field (gx, gy) of an H x W image into the image u whose
 * gradient is the least-squares fit of (gx, gy) on a zero-padded M x N torus
 * (Beaini et al., "Fast and Optimal Laplacian Solver for Gradient-Domain Image Editing
 * using Green Function Convolution", Sec. 2.2-2.3). In the paper's notation:
 *
 *   L   = div E, backward differences on the torus                      (eq. (3))
 *   G^  = F(dirac) / F(laplace) = 1/lambda,                             (eqs. (19)-(22),
 *         lambda(k,l) = -4 sin^2(pi k/M) - 4 sin^2(pi l/N), G^(0,0) = 0  Algorithm A)
 *   v   = R(F^-1(F(L) o G^))                                            (eq. (23))
 *   u   = v[block] - v[0,0]                                             (Algorithm B)
 *
 * The H x W block sits at offset (oy, ox) = (floor((M-H)/2), floor((N-W)/2)) of the torus
 * and the constant is fixed by the grid corner (0,0), which lies in the zero padding.
 *
 * Conventions for every entry point below:
 *  - Pointers named gx, gy, u, du, dgx, dgy are DEVICE pointers to float32 arrays laid out
 *    [B][H][W], row stride W, image stride H*W, contiguous. The caller owns them.
 *  - `workspace` is a DEVICE buffer of at least gfc_workspace_size() bytes, 256-byte
 *    aligned, owned by the caller. Its contents need not be initialised and are undefined
 *    after a call. Two calls that run concurrently need separate workspaces.
 *  - `stream` is a hipStream_t (NULL = the default stream). Solve calls only enqueue
 *    work: they never allocate, never synchronise the host and never copy host data. The
 *    forward column pass runs its few lowest-column tiles on a side stream owned by the
 *    plan, forked from and joined back to `stream` with events, so `stream` sees the
 *    call complete in order (graph capture follows the fork). Asynchronous kernel errors
 *    surface as GFC_E_HIP on a later call.
 *  - A plan owns its device tables (created by gfc_green_build) and is immutable after
 *    that call, so it may be used from several streams with separate workspaces, also
 *    from several host threads (the side-stream fork and join of a call are enqueued
 *    under a per-plan lock; the side stream serialises the low tiles of concurrent calls).
 *  - Errors are returned as status codes; nothing is ever thrown across this ABI.
 */
#ifndef GFC_H_
#define GFC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gfc_plan_s* gfc_plan_t;
typedef struct gfc_ragged_s* gfc_ragged_t;

typedef enum {
  GFC_OK = 0,
  GFC_E_ARG = 1,        /* null pointer, non-positive size, B < 0, bad flags           */
  GFC_E_SIZE = 2,       /* M < H+2 or N < W+2, or N has no supported row-FFT length      */
  GFC_E_NOT_BUILT = 3,  /* gfc_green_build has not run on this plan                      */
  GFC_E_WORKSPACE = 4,  /* workspace smaller than gfc_workspace_size()                   */
  GFC_E_HIP = 5,        /* a HIP runtime call or an earlier asynchronous kernel failed   */
  GFC_E_OOM = 6         /* device allocation of plan or schedule tables failed           */
} gfc_status;

/* Plan flags. */
#define GFC_FLAG_NONE 0u

/*
 * Create a plan for H x W images solved on an M x N torus (Sec. 2.3.2 zero padding).
 * M = N = 0 selects the default torus: the smallest even 2/3/5-smooth M >= max(2H, H + 2),
 * N >= max(2W, W + 2, 16) (16 is the shortest row FFT).
 * Requires M >= H + 2, N >= W + 2 and N a supported row-FFT length (even, 2/3/5-smooth,
 * listed by gfc_supported_length). Host-only: touches no GPU. *out receives the plan.
 */
gfc_status gfc_plan_create(gfc_plan_t* out, int H, int W, int M, int N, unsigned flags);

/*
 * Build the plan's device tables in float64 on the host and upload them on `stream`:
 * the row-FFT twiddles and, per column frequency l, the factorisation of the column
 * Green's function 1/lambda(., l) (eq. (22) restricted to one column of the spectrum).
 * Idempotent. Synchronises `stream` once (the only synchronising call besides destroy).
 */
gfc_status gfc_green_build(gfc_plan_t p, void* stream);

/*
 * Launch geometry of a plan (speed depends on it; results only through the summation
 * order of the float64 reference term over column tiles, "col_c"). Call before
 * gfc_green_build; GFC_E_ARG for an unknown name, a value out of range, or a built plan.
 *   "col_c"     1..64   (power of two) columns per workgroup in the column pass
 *   "col_rows"  16|32   rows per thread in the forward column pass
 *   "col_rows_b" 16|32  rows per thread in the backward column pass
 *   "low_bins"  4..32   K: row frequencies l <= K reach the forward column pass as the x-
 *                       and y-parts of the divergence separately (split form), 2K < N.
 *                       Changes the rounding, not the exact result: larger K costs a
 *                       direct-sum pass over the gradient for l in (4, K]. The default is
 *                       the smallest of 4, 8, 16, 32 with N <= 16 K M (thin, wide tori
 *                       get more: their solution is dominated by the lowest row bins).
 *   "row_split" N1   selects, among the row-transform entries compiled for N, the one whose
 *                    forward pass uses the split N = N1 x N2 (a library built for the
 *                    autotuner holds one entry per candidate split, every pass alike; the
 *                    default library holds one entry per N, GFC_E_ARG for any other N1)
 * The project's autotuner chooses the launch values per (H, W, M, N), and the split of each
 * row pass per row length (compiled into the default library); host-only.
 * gfc_plan_get_param also reads the fixed "low_bins_b" (Kb: backward columns l <= Kb take
 * -D_y inside the column recursion) and "row_split_fwd", "row_split_edit", "row_split_inv",
 * "row_split_bfwd", "row_split_binv": N1 of the split of the plain forward row pass, of its
 * other modes (edits, a given Laplacian, volume slices), and of the inverse, backward forward
 * and backward inverse row passes.
 */
gfc_status gfc_plan_set_param(gfc_plan_t p, const char* name, int value);
gfc_status gfc_plan_get_param(gfc_plan_t p, const char* name, int* value);

/* Resolved sizes of a plan: any output pointer may be NULL. */
gfc_status gfc_plan_get(gfc_plan_t p, int* H, int* W, int* M, int* N, int* oy, int* ox);

/* Bytes of workspace needed by gfc_solve_batch and gfc_solve_backward for B images. */
gfc_status gfc_workspace_size(gfc_plan_t p, int B, size_t* bytes);

/*
 * Forward solve of B images (eqs. (3), (22), (23) and Algorithm B):
 *   gx, gy : [B][H][W] float32 gradient fields (forward differences, eq. (1) convention)
 *   u      : [B][H][W] float32 output potential, u = v[block] - v[0,0]
 * B = 0 is a no-op. u must not alias gx or gy.
 */
gfc_status gfc_solve_batch(gfc_plan_t p, const float* gx, const float* gy, float* u, int B,
                           void* workspace, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): gfc_solve_batch with no workspace argument. The
 * workspace is a fixed array of GFC_NOALLOC_SCRATCH_BYTES inside the library, one copy per
 * GPU, held until the process ends; the call itself allocates nothing (its first call on a
 * GPU looks the array's device address up once). Same kernels and results as
 * gfc_solve_batch, bit for bit. GFC_E_WORKSPACE when the workspace of (p, B)
 * (gfc_workspace_size) exceeds GFC_NOALLOC_SCRATCH_BYTES, e.g. 801 x 1200 images on their
 * default torus take about 8.0 MiB each, so at most 7 per call. All calls on one GPU share
 * its array: calls that may overlap on one GPU (several streams or host threads) race on it
 * and must be serialised by the caller; calls in order on one stream are safe.
 */
#define GFC_NOALLOC_SCRATCH_BYTES (64u << 20)
gfc_status gfc_solve_batch_noalloc(gfc_plan_t p, const float* gx, const float* gy, float* u,
                                   int B, void* stream);

/*
 * Forward solve followed by the colour-preserving correction of eq. (25) (Sec. 3.2.2):
 *   u = (u_c - mean(u_c)) * I_std[b] / std(u_c) + I_mean[b]   over each H x W image,
 * where u_c is what gfc_solve_batch returns and I_mean, I_std ([B] float32, device) are the
 * mean and the population standard deviation of each source image I. The statistics of
 * u_c are float64 sums taken by the inverse row pass in a fixed order (deterministic); a
 * constant u_c (std 0) maps to I_mean. One more read and write of u than gfc_solve_batch.
 * Workspace as for gfc_solve_batch (gfc_workspace_size covers both).
 */
gfc_status gfc_solve_batch_color(gfc_plan_t p, const float* gx, const float* gy,
                                 const float* I_mean, const float* I_std, float* u, int B,
                                 void* workspace, size_t ws_bytes, void* stream);

/*
 * Forward solve from the Laplacian itself, Algorithm B's literal input:
 *   L : [B][H+1][W+1] float32, the divergence / Laplacian on the support of div E for H x W
 *       forward-difference fields (rows 0..H, columns 0..W of the image block; the Laplacian
 *       of an image whose first row and column are zero has exactly this support)
 *   u : [B][H][W] as for gfc_solve_batch.
 * L should sum to 0 (every divergence does): the torus solve cannot represent a net source,
 * and the DC column of L is integrated along y from row 0. Precision: the row bins l <= K
 * (the plan's "low_bins"), which the Green's function amplifies most, are not taken from the
 * float32 FFT of L: they are direct sums with float64 twiddles and accumulation, handed to
 * the column pass as running sums over the rows (a float64 scan), so that the sum over the
 * rows of each such bin is one rounded value rather than a difference of rounded values.
 */
gfc_status gfc_solve_laplacian(gfc_plan_t p, const float* L, float* u, int B, void* workspace,
                               size_t ws_bytes, void* stream);

/*
 * Gradient-domain editing in one call (Sec. 3.2): an edit of the gradient field, applied on
 * the device to each pixel as it is loaded, then the forward solve, then optionally the
 * colour correction of eq. (25).
 *   mode GFC_EDIT_THRESHOLD (Sec. 3.2.3): param = tau >= 0. A pixel's gradient is kept
 *     where fl(fl(gx*gx) + fl(gy*gy)) >= fl(tau*tau) (float32, in this order) and set to 0
 *     elsewhere. The paper thresholds at 10% of the highest possible gradient: tau is that
 *     absolute level. C is not read (may be NULL).
 *   mode GFC_EDIT_GDM (eq. (26)): param = alpha in [0, 1]; C [B][H][W] float32 >= 0 is the
 *     edge intensity. |E_p| = |E|^(1-alpha) * C^alpha with the orientation of E (float32
 *     log2/exp2); E_p = 0 where E = 0.
 *   I_mean, I_std: both NULL (no correction) or both [B] device arrays as for
 *     gfc_solve_batch_color.
 * GFC_E_ARG for an unknown mode, a parameter out of range, a missing C for GDM or only one
 * of I_mean, I_std. Workspace as for gfc_solve_batch. The edited field itself is never
 * stored; gx, gy and C are not modified.
 */
#define GFC_EDIT_THRESHOLD 1
#define GFC_EDIT_GDM 2
gfc_status gfc_solve_edit(gfc_plan_t p, const float* gx, const float* gy, const float* C,
                          int mode, float param, const float* I_mean, const float* I_std,
                          float* u, int B, void* workspace, size_t ws_bytes, void* stream);

/*
 * Backward (adjoint) of gfc_solve_batch, for using the solver as a differentiable layer
 * (Sec. 4): given du = dLoss/du [B][H][W], writes dgx = dLoss/dgx and dgy = dLoss/dgy:
 *   r = embed(du) - sum(du) * delta_(0,0);  w = g (*) r;
 *   dgx = -(w[y,x+1] - w[y,x]),  dgy = -(w[y+1,x] - w[y,x])   on the block,
 * where g is the spatial Green's function (real and even, so its correlation equals its
 * convolution). Outputs must not alias du.
 */
gfc_status gfc_solve_backward(gfc_plan_t p, const float* du, float* dgx, float* dgy, int B,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * Instrumentation: run one pass of gfc_solve_batch (stage 1 = row pass: divergence and row
 * transform; 2 = column pass: the Green's spectrum applied column by column; 3 = inverse
 * row pass with crop and constant; 0 = all three). Calling stages 1, 2, 3 in order on one
 * stream with one workspace is exactly gfc_solve_batch; it lets a caller time each kernel
 * with events between the passes. Arguments a stage does not read may be NULL.
 */
gfc_status gfc_solve_batch_stage(gfc_plan_t p, int stage, const float* gx, const float* gy,
                                 float* u, int B, void* workspace, size_t ws_bytes,
                                 void* stream);

/* Instrumentation: one pass of gfc_solve_backward (stages as for gfc_solve_batch_stage). */
gfc_status gfc_solve_backward_stage(gfc_plan_t p, int stage, const float* du, float* dgx,
                                    float* dgy, int B, void* workspace, size_t ws_bytes,
                                    void* stream);

/*
 * Tests only: write the plan's Green's spectrum G^ (eq. (22)) as float64 on the HOST,
 * half spectrum [M][N/2+1] row-major, G^(0,0) = 0. Host-only; needs no build.
 */
gfc_status gfc_green_export(gfc_plan_t p, double* half_spectrum_host);

void gfc_plan_destroy(gfc_plan_t p);

/* ---- ragged batches ---------------------------------------------------------------------
 * B images of different sizes solved together (each exactly as gfc_solve_batch would solve
 * it alone on its own torus). Inputs and outputs are PACKED: image i occupies elements
 * [off[i], off[i+1]) of gx, gy and u, row-major [H_i][W_i], off[0] = 0,
 * off[i+1] = off[i] + H_i * W_i (gfc_ragged_offsets). A ragged object owns one plan per
 * distinct image size (float64 tables built once) and a schedule of work items; its
 * solve replays a HIP graph captured on its first call.
 */

/* gfc_ragged_solve enqueues the passes directly instead of capturing and replaying a graph */
#define GFC_RAGGED_NO_GRAPH 1u

/*
 * Create a ragged object for B images: H[i] x W[i] on an M[i] x N[i] torus. M and N may be
 * NULL (or hold 0 entries) for the default torus of each image; the size rules are those
 * of gfc_plan_create, whose status is returned for the first image that breaks them.
 * flags: 0 or GFC_RAGGED_NO_GRAPH. Host-only.
 */
gfc_status gfc_ragged_create(gfc_ragged_t* out, int B, const int* H, const int* W,
                             const int* M, const int* N, unsigned flags);

/*
 * Build every image plan's float64 tables (as gfc_green_build), the per-image argument
 * tables and the work-item schedule, and upload them on `stream` (synchronises it once).
 * Idempotent.
 */
gfc_status gfc_ragged_build(gfc_ragged_t r, void* stream);

/* Resolved sizes of image i (any output may be NULL). Host-only. */
gfc_status gfc_ragged_image(gfc_ragged_t r, int i, int* H, int* W, int* M, int* N);

/* The B + 1 element offsets of the packed layout, written to a HOST array. */
gfc_status gfc_ragged_offsets(gfc_ragged_t r, int64_t* offsets);

/* Bytes of workspace needed by gfc_ragged_solve (after gfc_ragged_build). */
gfc_status gfc_ragged_workspace_size(gfc_ragged_t r, size_t* bytes);

/*
 * Forward solve of all B images (eqs. (3), (22), (23) and Algorithm B per image): gx, gy,
 * u are packed DEVICE arrays (see above); u must not alias gx or gy. The first call
 * captures the launch sequence into a HIP graph (host-side work); every call then writes
 * its buffer addresses into a device slot of the ragged object (a one-thread kernel on
 * `stream`) and launches the graph on `stream`, whose kernels read the addresses from that
 * slot. Any buffers may be passed on any call; the call never synchronises. With
 * GFC_RAGGED_NO_GRAPH every call enqueues the launches itself. Calls that may overlap
 * (other streams or threads) need separate ragged objects. Destroying the object waits for
 * the last launch of its graph.
 */
gfc_status gfc_ragged_solve(gfc_ragged_t r, const float* gx, const float* gy, float* u,
                            void* workspace, size_t ws_bytes, void* stream);

/*
 * The same result by B single-image gfc_solve_batch calls on `stream`, one per image with
 * its plan (the reference a ragged solve is compared against, and the plain baseline).
 */
gfc_status gfc_ragged_solve_sequential(gfc_ragged_t r, const float* gx, const float* gy,
                                       float* u, void* workspace, size_t ws_bytes,
                                       void* stream);

void gfc_ragged_destroy(gfc_ragged_t r);

/* 1 if N is a supported row-FFT length, else 0. Host-only. */
int gfc_supported_length(int N);

/* Human-readable status name. */
const char* gfc_status_str(gfc_status s);

/*
 * Volumes: three-dimensional GFC (the method holds in any dimension, eq. (5); the Green's
 * spectrum is 1/lambda with lambda = -4 sin^2(pi kz/P) - 4 sin^2(pi ky/M) - 4 sin^2(pi kx/N),
 * the 7-point stencil's symbol, and 0 at the DC bin). A D x H x W volume sits centred in a
 * P x M x N torus (P = 0: the smallest even 2/3/5-smooth P >= 2D, likewise M, N);
 * u = v[block] - v[0,0,0]. P is at most 512 and N a supported row length; M and N follow
 * gfc_plan_create's rules; one volume's spectra, P x (H+1) x (N/2+1, rounded up to a
 * multiple of 32) complex float32, stay below 2^31 bytes and one volume below 2^30 bytes
 * (GFC_E_SIZE otherwise).
 *   gx, gy, gz : [B][D][H][W] float32 forward-difference fields, zero exterior
 *   u          : [B][D][H][W] float32
 * Passes: rows of the 7-point divergence (x), whose 5 lowest row frequencies are kept as
 * the x-, y- and z-parts apart (direct sums of Ex, Ey, Ez); complex FFTs along z; the z
 * difference applied as its symbol to those bins; the column recursion along y per
 * (kz, l) with the y difference inside it; the inverse z FFT; the inverse rows with crop
 * and constant. Forward only. Errors and conventions as for the two-dimensional entry
 * points.
 */
typedef struct gfc_plan3_s* gfc_plan3_t;
gfc_status gfc_plan3_create(gfc_plan3_t* out, int D, int H, int W, int P, int M, int N,
                            unsigned flags);
gfc_status gfc_plan3_get(gfc_plan3_t p, int* D, int* H, int* W, int* P, int* M, int* N);
gfc_status gfc_green_build3(gfc_plan3_t p, void* stream);
gfc_status gfc_workspace3_size(gfc_plan3_t p, int B, size_t* bytes);
gfc_status gfc_solve3_batch(gfc_plan3_t p, const float* gx, const float* gy, const float* gz,
                            float* u, int B, void* workspace, size_t ws_bytes, void* stream);
void gfc_plan3_destroy(gfc_plan3_t p);

#ifdef __cplusplus
}
#endif
#endif /* GFC_H_ */
