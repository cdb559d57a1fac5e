/*
 * adorym.h -- C ABI of the MI355X multislice ptychography library.
 *
 * The library evaluates the far-field multislice forward model of the
 * paper's automatic-differentiation reconstruction framework and the
 * gradient of its data-mismatch loss:
 *
 *   y = F(x, theta),   L = D(y_meas, F(x, theta))
 *
 * (problem statement, Sec. 1, Eqs. forward_model / problem_equation /
 * loss_function), where x is the object (delta/beta refractive-index
 * decrements, Eq. ri_modulation, or real/imaginary transmission,
 * Eq. complex_modulation) and theta the probe and the per-position
 * subpixel shifts.  For each scan position the object chunk on the beam
 * path is gathered, the probe is placed by a Fourier shift
 * (Eq. fourier_shift), the wave is modulated by each slice and propagated
 * to the next with the paraxial Fresnel kernel (Eqs. fresnel_prop,
 * paraxial_kernel; multislice product, Sec. S1.C), and the exit wave is
 * taken to the detector with the Fraunhofer transform (Eq. fraunhofer);
 * Alg. 1 gives the order of these steps.  The loss is the LSQ amplitude
 * mismatch (Eq. lsq_loss) or the Poisson likelihood (Eq. poisson_loss).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer owned by the caller; the
 *    library never frees or retains it past the call.  Complex arrays are
 *    interleaved (re, im) float32 pairs.
 *  - Compute calls (forward, loss and gradient in every variant, priors,
 *    rotation, Adam, plan_run) are asynchronous on the context's stream
 *    and neither synchronise the host nor allocate device memory.  The
 *    set-up and measurement calls do, as each one's comment says:
 *    adorym_create / adorym_destroy, adorym_sync_error,
 *    adorym_plan_create / adorym_plan_destroy, adorym_loss_grad_batched,
 *    adorym_autotune, adorym_profile_start / adorym_profile_stop.
 *  - Host-checkable errors return at once and enqueue nothing.  Errors
 *    only the device can see (a chunk that leaves the object) set a
 *    sticky flag read by adorym_sync_error; the offending positions
 *    contribute nothing (zero intensity, zero gradient, zero loss).
 *  - Object arrays are slice-major planar float32 [S][Ly][Lx]; element
 *    (j, y, x) is at j*Ly*Lx + y*Lx + x.
 *  - Positions: int32 corners [B][2] (y, x) of the N x N chunk in object
 *    pixels, and float32 residual shifts [B][2] (y, x) in pixels.  The
 *    probe is shifted so that p_b(r) = p(r - s) (periodic).  A float
 *    position r is passed as corner floor(r + 0.5) and shift r - corner.
 *  - The FFT convention: unitary transforms; the far field is the
 *    positive-exponent (inverse) DFT of the exit wave, centred so that the
 *    zero frequency lies at (N/2, N/2) of the [N][N] detector array.
 *  - S slices give S - 1 inter-slice propagations by the slice spacing.
 *  - Loss = mean over the B*N*N detector pixels of the call; eps is added
 *    inside both square roots (LSQ) and inside the logarithm (Poisson).
 *  - Complex gradients are dL/dRe + i dL/dIm.
 */
#ifndef ADORYM_H
#define ADORYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adorym_ctx adorym_ctx;

typedef enum {
  ADORYM_OK = 0,
  ADORYM_EINVAL = 1,        /* bad argument (null pointer, size < 1, ...)         */
  ADORYM_EUNSUPPORTED = 2,  /* e.g. a probe size N the library has no kernel for  */
  ADORYM_ERANGE = 3,        /* a chunk left the object (device-detected, deferred) */
  ADORYM_ENOMEM = 4,        /* workspace smaller than adorym_workspace_size        */
  ADORYM_EDEVICE = 5        /* a HIP runtime call failed                           */
} adorym_status;

enum { ADORYM_LOSS_GAUSSIAN = 0, ADORYM_LOSS_POISSON = 1 };
enum { ADORYM_OBJ_DELTA_BETA = 0, ADORYM_OBJ_REAL_IMAG = 1 };
enum { ADORYM_PROP_PARAXIAL = 0, ADORYM_PROP_SOMMERFELD = 1 };   /* near-field detector kernels */
enum {
  ADORYM_ACCUMULATE_GRADS = 1u, /* add into the gradient arrays instead of overwriting */
  ADORYM_DETERMINISTIC = 2u     /* bitwise-reproducible object gradients (see below)  */
};
/* Gradient accumulation.  Each position stores its contribution to
 * dL/d(object) in the workspace (B*S*2*N*N*4 bytes, no atomics) and a second
 * kernel sums, for every voxel, the contributions of the positions in index
 * order in FP64, rounding once to float32; loss, probe and shift gradients
 * are also reduced in a fixed order.  Every call is therefore reproducible
 * bit for bit for a given split.  ADORYM_DETERMINISTIC additionally fixes
 * the split per probe size (k = 1 for N <= 96, 4 for N = 128, 6 for
 * N = 192; adorym_set_split does not apply), so that results are also the
 * same bits between a single call and the same job inside a batched plan
 * next to other jobs, whatever split other calls use. */

/* Geometry and options of one scan. */
typedef struct {
  int32_t n;            /* probe / chunk / detector size N (N x N)                 */
  int32_t n_slices;     /* S >= 1                                                  */
  int32_t obj_ny;       /* Ly                                                      */
  int32_t obj_nx;       /* Lx                                                      */
  double wavelength_m;  /* lambda; k = 2 pi / lambda                               */
  double pixel_m;       /* lateral pixel size dx (Fresnel kernel frequencies)      */
  double slice_dz_m;    /* slice spacing dz (Fresnel distance and k dz)            */
  int32_t loss;         /* ADORYM_LOSS_*                                           */
  int32_t obj_repr;     /* ADORYM_OBJ_*                                            */
  int32_t ckpt_every;   /* slice checkpoint interval C (>= 1; 16 is typical)       */
  double eps;           /* loss epsilon (photons)                                  */
  uint32_t flags;       /* ADORYM_ACCUMULATE_GRADS | ADORYM_DETERMINISTIC          */
} adorym_geom;

/* Create a context on HIP device `device` issuing work on `stream`
 * (a hipStream_t; NULL = the null stream).  Allocates a few bytes of
 * device memory for the deferred error flag. */
adorym_status adorym_create(adorym_ctx** out, int device, void* stream);
adorym_status adorym_destroy(adorym_ctx* ctx);
/* Change the stream later calls are enqueued on. */
adorym_status adorym_set_stream(adorym_ctx* ctx, void* stream);

/* Probe sizes with a kernel: returns 1 if N is supported. */
int adorym_supports_n(int32_t n);

/* Bytes of device workspace adorym_loss_grad needs for a batch of `batch`
 * positions (probe spectrum, per-position loss, shift and probe partials,
 * slice checkpoints every ckpt_every slices, room for the waves of one
 * checkpoint segment per position, the exchange buffers of split
 * workgroups and the staged object-gradient contributions).  0 on bad
 * input.
 *
 * The reverse sweep rebuilds the wave entering each slice by dividing the
 * next one by the slice's transmission, re-anchored on the checkpoints.
 * Before each loss-and-gradient evaluation a pre-pass bounds, per slice, the
 * largest -log|t| of its voxels (k dz beta, or -log|O|); a checkpoint
 * segment whose slices could amplify rounding by more than 2^4 that way
 * (strong absorbers, or a transmission of exactly zero) has its waves
 * recomputed forward from its checkpoint instead, so any object gives
 * finite gradients at float32 accuracy; such segments cost about half a
 * forward sweep more. */
size_t adorym_workspace_size(const adorym_geom* g, int32_t batch);
/* The smaller workspace adorym_forward needs (probe spectrum, exchange
 * buffers and counters only); adorym_workspace_size also suffices. */
size_t adorym_forward_workspace_size(const adorym_geom* g, int32_t batch);

/* Forward model (Alg. 1 without refinement of anything): predicted
 * far-field intensities |Psi|^2, float32 [B][N][N], zero frequency at
 * (N/2, N/2).  obj_a/obj_b: delta/beta or real/imag [S][Ly][Lx];
 * probe complex [N][N].  Workspace of adorym_forward_workspace_size bytes. */
adorym_status adorym_forward(adorym_ctx* ctx, const adorym_geom* g,
                             const float* obj_a, const float* obj_b, const float* probe,
                             const int32_t* corner, const float* shift, int32_t batch,
                             float* intensity, void* workspace, size_t ws_bytes);

/* adorym_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): the workspace is a static device
 * array of 64 MiB that the library holds on every GPU it runs on until the
 * process ends, located at adorym_create.  The call itself allocates
 * nothing.  Inputs and the output are the caller's, as for adorym_forward.
 * ADORYM_ENOMEM (nothing enqueued) when adorym_forward_workspace_size(g,
 * batch) exceeds 64 MiB, e.g. more than 127 positions at N = 128.  Every
 * call on one GPU uses that GPU's one array: calls that overlap on the
 * device (other streams, other contexts, other threads) race and must be
 * ordered by the caller.  Results equal adorym_forward's bit for bit. */
adorym_status adorym_forward_static(adorym_ctx* ctx, const adorym_geom* g,
                                    const float* obj_a, const float* obj_b, const float* probe,
                                    const int32_t* corner, const float* shift, int32_t batch,
                                    float* intensity);

/* Loss and gradient.  i_meas float32 [B][N][N] (zero frequency at N/2).
 * Writes *loss (device double), and, for every gradient pointer that is
 * not NULL: g_a/g_b [S][Ly][Lx] (dL/ddelta, dL/dbeta or dL/dRe O, dL/dIm O),
 * g_probe complex [N][N], g_shift [B][2] (dL/ds, equal to dL/dr).
 * Gradients overwrite unless ADORYM_ACCUMULATE_GRADS is set.  `intensity`
 * may be NULL; if given, the predicted intensities are written too. */
adorym_status adorym_loss_grad(adorym_ctx* ctx, const adorym_geom* g,
                               const float* obj_a, const float* obj_b, const float* probe,
                               const int32_t* corner, const float* shift, int32_t batch,
                               const float* i_meas, void* workspace, size_t ws_bytes,
                               double* loss, float* g_a, float* g_b, float* g_probe,
                               float* g_shift, float* intensity);

/* ---- Probe defocus (a refinable parameter of the experiment, Sec. S1.D) --
 * The probe is Fresnel-propagated by defocus_m metres (host double, any
 * finite value; Eqs. fresnel_prop, paraxial_kernel: its spectrum times
 * exp(i pi lambda defocus_m |nu|^2)) before it meets the object; `probe` is
 * the undefocused probe.  adorym_forward_defocus: as adorym_forward, same
 * workspace.  adorym_loss_grad_defocus: as adorym_loss_grad, same
 * workspace; g_probe is the gradient with respect to the undefocused probe
 * and, if g_defocus (DEVICE float64 scalar) is not NULL, it receives
 * dL/d(defocus_m) in 1/m (overwritten, or added with
 * ADORYM_ACCUMULATE_GRADS), summed in FP64 in a fixed order.  A non-finite
 * defocus_m is ADORYM_EINVAL.  defocus_m = 0 gives the plain calls' bits. */
adorym_status adorym_forward_defocus(adorym_ctx* ctx, const adorym_geom* g,
                                     const float* obj_a, const float* obj_b, const float* probe,
                                     const int32_t* corner, const float* shift, int32_t batch,
                                     double defocus_m, float* intensity, void* workspace, size_t ws_bytes);
adorym_status adorym_loss_grad_defocus(adorym_ctx* ctx, const adorym_geom* g,
                                       const float* obj_a, const float* obj_b, const float* probe,
                                       const int32_t* corner, const float* shift, int32_t batch,
                                       double defocus_m, const float* i_meas, void* workspace, size_t ws_bytes,
                                       double* loss, float* g_a, float* g_b, float* g_probe,
                                       float* g_shift, double* g_defocus, float* intensity);

/* ---- Unequal slice spacing: sparse multislice (Sec. S1.C, the variable-
 * spacing variant; slice positions are refinable parameters, Sec. S1.D) ---
 * gaps: DEVICE float64 [S-1], gaps[j] = free-space distance (metres) from
 * slice j to slice j+1, replacing slice_dz_m in the Fresnel kernel of that
 * gap (H_j = exp(i pi lambda gaps[j] |nu|^2)); slice_dz_m keeps its role as
 * the slice thickness in the transmission exp(i k dz delta - k dz beta).
 * Any real value is accepted (zero: adjacent slices act as one thin
 * object; negative: back-propagation).  May be NULL when S == 1.
 * adorym_forward_gaps: as adorym_forward, workspace of
 * adorym_forward_workspace_size bytes.
 * adorym_loss_grad_gaps: as adorym_loss_grad, workspace of
 * adorym_gaps_workspace_size bytes, and, if g_gaps (DEVICE float64 [S-1])
 * is not NULL, dL/d(gaps[j]) in 1/m (overwritten, or added with
 * ADORYM_ACCUMULATE_GRADS).  The gap gradient of each position is reduced
 * in FP64 in a fixed order.  Both run with one fixed split per probe size
 * (1 for N <= 96, 4 for N = 128, 6 for N = 192), whatever adorym_set_split
 * chose. */
size_t adorym_gaps_workspace_size(const adorym_geom* g, int32_t batch);
adorym_status adorym_forward_gaps(adorym_ctx* ctx, const adorym_geom* g,
                                  const float* obj_a, const float* obj_b, const float* probe,
                                  const int32_t* corner, const float* shift, int32_t batch,
                                  const double* gaps, float* intensity, void* workspace, size_t ws_bytes);
adorym_status adorym_loss_grad_gaps(adorym_ctx* ctx, const adorym_geom* g,
                                    const float* obj_a, const float* obj_b, const float* probe,
                                    const int32_t* corner, const float* shift, int32_t batch,
                                    const double* gaps, const float* i_meas, void* workspace, size_t ws_bytes,
                                    double* loss, float* g_a, float* g_b, float* g_probe,
                                    float* g_shift, double* g_gaps, float* intensity);

/* ---- Near field: Fresnel propagation to the detector (holography,
 * near-field ptychography; Eq. fresnel_prop with Eq. paraxial_kernel or
 * Eq. sommerfeld_kernel; free propagation distance refinement, Sec. S1.D)
 * In place of the Fraunhofer transform the exit wave is propagated over the
 * distance dist[dist_idx[b]] to the detector: I = |F^-1[H F phi_exit]|^2,
 * natural (not centred) order, float32 [B][N][N].
 * kind: ADORYM_PROP_PARAXIAL, H = exp(i pi lambda d |nu|^2), or
 * ADORYM_PROP_SOMMERFELD, H = exp(-i k d sqrt(1 - lambda^2 |nu|^2)) with the
 * evanescent frequencies (lambda |nu| >= 1) removed; its global phase
 * exp(-i k d) is left out (no effect on intensities or their gradients).
 * dist: DEVICE float64 [n_dist] metres (any sign); dist_idx: DEVICE int32
 * [B], each in [0, n_dist) (a position with another index contributes
 * nothing and adorym_sync_error reports ADORYM_EINVAL).
 * adorym_loss_grad_nearfield also writes, if g_dist (DEVICE float64
 * [n_dist]) is not NULL, dL/d(dist[d]) summed over the positions with that
 * index (overwritten, or added with ADORYM_ACCUMULATE_GRADS), reduced in
 * FP64 in a fixed order.  Workspace of adorym_nearfield_workspace_size
 * bytes for both calls.  Both run with the fixed split of
 * ADORYM_DETERMINISTIC (1 for N <= 96, 4 for N = 128, 6 for N = 192). */
size_t adorym_nearfield_workspace_size(const adorym_geom* g, int32_t batch, int32_t n_dist);
adorym_status adorym_forward_nearfield(adorym_ctx* ctx, const adorym_geom* g,
                                       const float* obj_a, const float* obj_b, const float* probe,
                                       const int32_t* corner, const float* shift, int32_t batch,
                                       int32_t kind, const double* dist, int32_t n_dist,
                                       const int32_t* dist_idx, float* intensity,
                                       void* workspace, size_t ws_bytes);
adorym_status adorym_loss_grad_nearfield(adorym_ctx* ctx, const adorym_geom* g,
                                         const float* obj_a, const float* obj_b, const float* probe,
                                         const int32_t* corner, const float* shift, int32_t batch,
                                         int32_t kind, const double* dist, int32_t n_dist,
                                         const int32_t* dist_idx, const float* i_meas,
                                         void* workspace, size_t ws_bytes, double* loss, float* g_a,
                                         float* g_b, float* g_probe, float* g_shift, double* g_dist,
                                         float* intensity);

/* ---- Several mutually incoherent probe modes (Eq. multimode) ----------
 * The detector records the sum over modes m of |Psi_m|^2, each mode
 * propagated through the same object at the same positions; the loss is the
 * one of adorym_loss_grad evaluated at that summed intensity.
 * probes: complex [M][N][N].  Outputs as adorym_loss_grad, except g_probe
 * complex [M][N][N] (one gradient per mode) and `intensity`, if given, the
 * summed intensity.  g_a, g_b and g_shift are sums over the modes.
 * Runs M forward passes, each keeping its slice checkpoints and exit waves
 * and adding its intensity into the sum, then M loss-and-gradient passes
 * that resume from what their forward pass kept (no second forward sweep),
 * all on the context's stream, with the fixed split of ADORYM_DETERMINISTIC
 * (1 for N <= 96, 4 for N = 128, 6 for N = 192).  Workspace of
 * adorym_modes_workspace_size(g, batch, M) bytes: one adorym_loss_grad
 * workspace, two intensity planes [B][N][N] and per mode the checkpoints
 * and exit waves.  With M = 1 the results equal, bit for bit, those of
 * adorym_loss_grad with ADORYM_DETERMINISTIC. */
size_t adorym_modes_workspace_size(const adorym_geom* g, int32_t batch, int32_t n_modes);
adorym_status adorym_loss_grad_modes(adorym_ctx* ctx, const adorym_geom* g,
                                     const float* obj_a, const float* obj_b, const float* probes,
                                     int32_t n_modes, const int32_t* corner, const float* shift,
                                     int32_t batch, const float* i_meas, void* workspace, size_t ws_bytes,
                                     double* loss, float* g_a, float* g_b, float* g_probe,
                                     float* g_shift, float* intensity);

/* Loss now, gradients later (a torch.autograd.Function's forward and
 * backward).  adorym_loss_fwd runs the forward model, keeps every
 * position's slice checkpoints and exit wave in the workspace (of
 * adorym_loss_fwd_workspace_size bytes), writes *loss (device double) and,
 * if `intensity` is not NULL, the predicted intensities.  adorym_loss_bwd,
 * called later with the same arguments and the untouched workspace, resumes
 * from what the forward kept (no second forward sweep) and writes the
 * gradients of grad_scale * L (grad_scale a finite float32 value; the
 * reverse sweep is linear in it).  Gradient pointers and
 * ADORYM_ACCUMULATE_GRADS as in adorym_loss_grad.  Both run with the fixed
 * split of ADORYM_DETERMINISTIC, except at N = 128 with more than 128
 * positions and without that flag, where they use one workgroup per
 * position, the split adorym_loss_grad chooses there unless adorym_set_split
 * overrides it.  With grad_scale = 1 the gradients equal, bit for bit, those
 * of adorym_loss_grad run with the same split. */
size_t adorym_loss_fwd_workspace_size(const adorym_geom* g, int32_t batch);
adorym_status adorym_loss_fwd(adorym_ctx* ctx, const adorym_geom* g,
                              const float* obj_a, const float* obj_b, const float* probe,
                              const int32_t* corner, const float* shift, int32_t batch,
                              const float* i_meas, void* workspace, size_t ws_bytes,
                              double* loss, float* intensity);
adorym_status adorym_loss_bwd(adorym_ctx* ctx, const adorym_geom* g,
                              const float* obj_a, const float* obj_b, const float* probe,
                              const int32_t* corner, const float* shift, int32_t batch,
                              const float* i_meas, void* workspace, size_t ws_bytes, double grad_scale,
                              float* g_a, float* g_b, float* g_probe, float* g_shift);

/* Tilt rotation of a slice-major float32 object [lz][ly][lx] about the y
 * axis (Sec. S1.D.2, Eq. rotation_transform): every xz-plane is resampled
 * by bilinear interpolation at (x0, z0) = R(theta)(x_t - cx, z_t - cz) + c,
 * c = ((lx-1)/2, (lz-1)/2), zero outside.  transpose = 0: out = R in;
 * transpose = 1: out = R^T in, the exact adjoint (for gradients).  `out` is
 * overwritten and must not alias `in`.  Coordinates are computed in FP64. */
adorym_status adorym_rotate(adorym_ctx* ctx, const float* in, float* out, int32_t lz, int32_t ly, int32_t lx,
                            double theta, int transpose);

/* ---- Object priors (Eq. tikhonov, Table tab:regularizers) -------------
 * Regularizers added to the data loss, on the object [S][Ly][Lx] (DEVICE
 * float32 obj_a/obj_b as in adorym_loss_grad).  With N_o = S Ly Lx voxels
 * and the per-voxel quantities q1, q2 = (delta, beta) for
 * ADORYM_OBJ_DELTA_BETA or (|O| - mean|O|, arg O) for ADORYM_OBJ_REAL_IMAG:
 *   R = (1/N_o) sum [l1_a W1 |q1| + l1_b W2 |q2|]                (l1)
 *     + (tv/N_o) sum over neighbouring voxel pairs along z, y, x
 *       of |q1' - q1| + |q2' - q2|                                (TV)
 * W1, W2 = 1, or the reweighted-l1 weights w_a, w_b (DEVICE float32, same
 * shape, both or neither).  The derivative of |t| at 0 is taken as 0;
 * mean|O| is differentiated through.
 * adorym_prior_grad: writes R to *value (DEVICE float64) and adds dR/da,
 * dR/db onto g_a, g_b (accumulate != 0, the usual case after
 * adorym_loss_grad) or overwrites them (accumulate == 0).  Coefficients
 * must be >= 0.  Workspace of adorym_prior_workspace_size bytes.  All sums
 * are in FP64 in a fixed order.
 * adorym_prior_weights: W = max|q| / (|q| + eps) per voxel from a snapshot
 * of the object (the adaptive weights of the reweighted l1, held constant
 * between updates), eps > 0.
 * adorym_support_project: the finite-support constraint: voxels whose mask
 * byte (DEVICE uint8 [n]) is 0 are set to vacuum (delta = beta = 0, or
 * O = 1 + 0i), in place. */
size_t adorym_prior_workspace_size(int32_t s, int32_t ly, int32_t lx);
adorym_status adorym_prior_grad(adorym_ctx* ctx, int32_t obj_repr, const float* obj_a, const float* obj_b,
                                int32_t s, int32_t ly, int32_t lx, double l1_a, double l1_b, double tv,
                                const float* w_a, const float* w_b, void* workspace, size_t ws_bytes,
                                double* value, float* g_a, float* g_b, int32_t accumulate);
adorym_status adorym_prior_weights(adorym_ctx* ctx, int32_t obj_repr, const float* snap_a, const float* snap_b,
                                   int32_t s, int32_t ly, int32_t lx, double eps, void* workspace,
                                   size_t ws_bytes, float* w_a, float* w_b);
adorym_status adorym_support_project(adorym_ctx* ctx, int32_t obj_repr, const uint8_t* mask, float* obj_a,
                                     float* obj_b, size_t n);

/* One Adam step (Sec. S1.F) on n float32 values, in place on x, m, v:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * x -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t >= 1.
 * Complex arrays are updated as independent real and imaginary parts. */
adorym_status adorym_adam(adorym_ctx* ctx, float* x, const float* g, float* m, float* v, size_t n, double lr,
                          double beta1, double beta2, double eps, int32_t t);
/* The same Adam step with the iteration count t read from DEVICE memory
 * (int32 scalar) when the kernel runs, so that a HIP graph holding the whole
 * iteration (loss, gradients and this step) uses the current count on
 * every replay; the caller advances *t between iterations (inside the graph
 * too).  A count below 1 leaves x, m and v unchanged and makes
 * adorym_sync_error report ADORYM_EINVAL. */
adorym_status adorym_adam_dev(adorym_ctx* ctx, float* x, const float* g, float* m, float* v, size_t n, double lr,
                              double beta1, double beta2, double eps, const int32_t* t);

/* ---- Batched evaluation of many independent scans --------------------
 * One job = the arguments of one adorym_loss_grad call (its own geometry,
 * object, probe, positions, measurements, outputs and workspace of
 * adorym_workspace_size(&g, batch) bytes).  adorym_plan_create validates the
 * jobs and uploads a job table (it allocates and synchronises: call it
 * outside timed or captured regions; it also creates the plan's own
 * streams).  adorym_plan_run then evaluates every job's loss and gradients:
 * per probe size, one persistent launch whose workgroup groups draw (job,
 * position) items from a device queue, longest first.  Sizes split over
 * several workgroups run first on ctx's stream; sizes with one workgroup
 * per position then run concurrently on the plan's streams, forked from
 * and joined back to ctx's stream by events.  It only launches kernels and
 * records and waits on events, so a whole iteration can be captured in a
 * HIP graph.  The arrays named in the jobs must stay valid while the plan
 * is used.  Supported probe sizes as adorym_supports_n. */
typedef struct {
  adorym_geom g;
  const float* obj_a; const float* obj_b; const float* probe;
  const int32_t* corner; const float* shift; int32_t batch;
  const float* i_meas;
  double* loss; float* g_a; float* g_b; float* g_probe; float* g_shift;
  void* workspace; size_t ws_bytes;
  float* intensity;     /* predicted intensities [B][N][N], or NULL: not written */
} adorym_job;
typedef struct adorym_plan adorym_plan;
adorym_status adorym_plan_create(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs, adorym_plan** out);
/* One-shot batched evaluation: plan_create, plan_run, a stream
 * synchronisation and plan_destroy (it allocates and synchronises; for
 * repeated iterations keep a plan). */
adorym_status adorym_loss_grad_batched(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs);
/* Autotuner of the split per probe size: for every probe size among the
 * jobs (deterministic jobs excepted: their split is fixed) it times `reps`
 * plan runs of those jobs with each supported split (N = 64: 1, 2, 4;
 * 96: 1, 2, 3, 4; 128: 1, 2, 4, 8; 192: 2, 4, 6, 8), keeps the fastest and
 * sets it on the context (as adorym_set_split).  chosen, if not NULL,
 * receives the split for N = 64, 96, 128, 192 (the context's current
 * value, 0 = automatic, for sizes without jobs).  The jobs' outputs are
 * overwritten.  Allocates and synchronises: a set-up call. */
adorym_status adorym_autotune(adorym_ctx* ctx, const adorym_job* jobs, int32_t n_jobs, int32_t reps,
                              int32_t* chosen);
/* Runs every job of the plan on ctx's stream (kernel launches only). */
adorym_status adorym_plan_run(adorym_ctx* ctx, adorym_plan* plan);
/* Frees the plan's device tables (hipFree: waits for the device); NULL is
 * EINVAL.  Call it only after the plan's last run has completed. */
adorym_status adorym_plan_destroy(adorym_plan* plan);

/* Synchronise the context's stream, return (and clear) any deferred
 * device-side error, e.g. ADORYM_ERANGE. */
adorym_status adorym_sync_error(adorym_ctx* ctx);

/* Human-readable description of the last error on this context. */
const char* adorym_last_error_message(adorym_ctx* ctx);

/* Number of workgroups that share one position's wavefield for probe size
 * n: k = 1 keeps the field in one workgroup (transposes through LDS);
 * k > 1 splits its lines over k workgroups that exchange through L2.
 * k = 0 restores the automatic choice (enough workgroups to cover the
 * CUs).  Supported: n = 64 with k in {1, 2, 4}; n = 96 with k in
 * {1, 2, 3, 4}; n = 128 with k in {1, 2, 4, 8}; n = 192 with k in
 * {2, 4, 6, 8} (its field does not fit one workgroup); else
 * ADORYM_EUNSUPPORTED.  Results do not depend on k
 * beyond float rounding of the gradient atomics. */
adorym_status adorym_set_split(adorym_ctx* ctx, int32_t n, int32_t k);

/* Kernel timing for benchmarks.  adorym_profile_start creates up to
 * max_launches pairs of HIP events (it allocates: call it outside a timed
 * region); while enabled, every forward / loss_grad call records one pair
 * around its main multislice kernel on the context's stream.
 * adorym_profile_stop synchronises the stream and returns the summed
 * kernel time in milliseconds and the number of timed launches. */
adorym_status adorym_profile_start(adorym_ctx* ctx, int32_t max_launches);
adorym_status adorym_profile_stop(adorym_ctx* ctx, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* ADORYM_H */
