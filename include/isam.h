/*
 * isam.h -- C ABI of the MI355X full-range ISAM operator and its FISTA solve.
 *
 * Model (arXiv 1905.06058, Mason, Davies & Bagnaninchi):
 *   real spectra   s = Re(K^ eta)                         (Eq. 5, 8)
 *   operator       K^ = diag(e^{j phi}) K                 (Eq. 13)
 *                  K  = F_<->^{-1} diag(b) N F_<->         (Eq. 16)
 *   back-projection K^H s = N'(F_<->(s))                   (Eq. 17)
 *   MBIR problem   argmin 1/2 ||Re(K^ eta) - s_d||^2 + lambda w^T |eta|   (Eq. 12)
 *   solver         FISTA with the weighted complex soft threshold          (Alg. 1, Eq. 14, 15)
 *
 * F_<-> is the unitary lateral DFT (exp(-2 pi i l p / nx) / sqrt(nx)).  N is the
 * Stolt resampling of Eq. 3: for lateral frequency q_l and wavenumber k_n it
 * evaluates the object's depth spectrum at kz = sqrt(4 k_n^2 - q_l^2),
 *   X[l][n] = nz^{-1/2} sum_m eta_hat[l][m] exp(+i kz z_m),
 * through a min-max NUFFT (Kaiser-Bessel scaling, 2x oversampled FFT, J = 6
 * interpolation taps).  b and the focus are folded into the pointwise factor
 *   c[l][n] = B(q_l) e^{j phi(k_n)} e^{j (2 k_n - kz) z_f},
 *   B(q) = exp(-q^2 w0^2 / 8) on propagating components (q^2 < 4k^2), else 0,
 *   phi(k) = a2 (k - k0)^2 + a3 (k - k0)^3,  k0 = 2 pi / lambda_c  (Eq. 7).
 *
 * Sampling: nk samples uniform in k over the band 2 pi dlambda / lambda_c^2
 * centred on k0; the full-range depth grid has nz = nk rows of pitch
 * pi / band, row m in [-nz/2, nz/2) stored at depth index i = m + nz/2.
 *
 * Volumes (ny > 1, the 3-D form N = nx ny nz of Sec. "Background"): the lateral
 * DFT runs over both lateral axes, q^2 = qx^2 + qy^2, and every (qx, qy) column
 * gets the same Stolt NUFFT.
 *
 * Layouts (all row-major, caller-owned device memory):
 *   object eta    complex64 interleaved (re, im) float pairs, [ny][nx][nk], depth contiguous
 *   spectra s, y  float32 [ny][nx][nk], k contiguous
 *   weights w     float32 [ny][nx][nk] (same layout as eta), or NULL for w = 1
 * (ny = 1 for a B-scan: [nx][nk].)  Shapes written [nx][nk] below mean [ny][nx][nk]
 * for a volume.
 *
 * Every entry point returns ISAM_OK (0) or a negative ISAM_E* code; none aborts
 * or throws.  Work is enqueued on the given HIP stream (a hipStream_t passed as
 * void*, NULL = the null stream) and is asynchronous unless stated otherwise.
 * Device pointers must stay valid until the stream has completed the work.
 * A plan owns its tables and workspace; one plan must not be used on two
 * streams at the same time (calls on one plan are stream-ordered).
 */
#ifndef ISAM_H
#define ISAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISAM_OK = 0,
    ISAM_EINVAL = -1,        /* bad argument: null pointer, size or non-finite optics */
    ISAM_EALIAS = -2,        /* an output aliases an input */
    ISAM_EUNSUPPORTED = -3,  /* valid but not built: J != 6, osf != 2; nk not a power of two or
                                above 4096; nx or ny not a built lateral length (powers of two up
                                to 2048; 192, 320, 384, 448, 640, 768, 896, 1280, 1536, 1792);
                                more than 2^30 object samples; Stolt positions that break the
                                adjoint's slot bounds (see isam_plan) */
    ISAM_ENOMEM = -4,        /* device allocation failed */
    ISAM_ENODEV = -5,        /* no HIP device visible */
    ISAM_EHIP = -6,          /* a HIP runtime call failed */
    ISAM_ENONFINITE = -7     /* FISTA met a non-finite norm (NaN/Inf in the data or divergence) */
};

typedef struct isam_plan_s* isam_plan_t;

/* Geometry of one B-scan or volume (SI units).  Sec. "Background" fixes
 * N = nx ny nz with nz the spectrometer length; Eq. 3 the Stolt map; Eq. 7 the
 * dispersion. */
typedef struct {
    int32_t nx, ny, nk;      /* A-scans per row, rows (1 for a B-scan), spectral samples (= depth rows) */
    double dx, dy;           /* lateral pitches [m] (dy unused when ny = 1) */
    double lambda_c;         /* centre wavelength [m] */
    double dlambda;          /* bandwidth [m]; sampling is uniform in k */
    double waist;            /* Gaussian beam waist w0 [m] of the beam filter B */
    double z_focus;          /* focal depth from zero delay [m] (any real value) */
    double a2, a3;           /* dispersion coefficients of Eq. 7 [rad m^2], [rad m^3]; a1 = 0 */
    int32_t J;               /* NUFFT interpolation taps (6) */
    int32_t osf;             /* NUFFT oversampling factor (2) */
    double kb_beta;          /* Kaiser-Bessel scaling shape; <= 0 selects 2.34 J */
} isam_geometry;

/* Result record of isam_fista. */
typedef struct {
    int32_t iters_run;       /* iterations executed */
    int32_t status;          /* 0, or ISAM_ENONFINITE */
    double rel_res;          /* relative residual r_r of Eq. 15 at the last iteration (tol > 0 only, else -1) */
    double resid2;           /* ||A eta^k - y||^2 at the last iteration's momentum point */
    double l1;               /* sum_i w_i |z_i| of the returned iterate (before residual add-back) */
    double L;                /* step constant used (1/L is the gradient step) */
} isam_fista_info;

/* Create a plan for geometry *g: the sampling of Sec. "Background" (N = nx ny nz,
 * nz = nk), the Stolt map of Eq. 3 and the dispersion of Eq. 7, evaluated through the
 * min-max NUFFT the paper adopts (Sec. "Efficient and robust ISAM through non-uniform
 * FFT").  Validates, allocates tables and workspace, and builds the tables in FP64 on
 * the device (Stolt constants, beam filter, dispersion and focus phases, Kaiser-Bessel
 * scaling, the min-max weight table, FFT twiddles).  Then it checks on the device, with
 * the kernels' own FP64 Stolt arithmetic, the two bounds that the adjoint's atomic-free
 * transposed interpolation relies on (consecutive samples of a column at least two
 * oversampled cells apart; a chunk of samples within its slot array); a geometry that
 * breaks them gets EUNSUPPORTED.  At q = 0 the Stolt map is the identity and the
 * positions advance by exactly two cells per sample.  Synchronises `stream`.
 * *out receives the plan (NULL on error).  Errors: EINVAL, EUNSUPPORTED,
 * ENODEV, ENOMEM, EHIP. */
int isam_plan(const isam_geometry* g, void* stream, isam_plan_t* out);

/* Change the calibration (a2, a3, z_focus) of an existing plan and rebuild the
 * tables that depend on it (Eq. 7 and the focal reference); same sizes.
 * Stream-ordered after earlier work on `stream`; synchronises it at the end. */
int isam_set_calibration(isam_plan_t p, double a2, double a3, double z_focus, void* stream);

/* Forward operator s_out = Re(K^ eta) (Eq. 5, 13, 16).
 * eta: device complex64 [nx][nk]; s_out: device float32 [nx][nk]; must not alias.
 * Three kernels: lateral FFT, Stolt NUFFT per lateral-frequency pair, lateral
 * C2R inverse FFT.  Errors: EINVAL (null), EALIAS. */
int isam_forward(isam_plan_t p, const void* eta, float* s_out, void* stream);

/* Adjoint eta_out = K^^H r (Eq. 17): the adjoint of isam_forward under the real
 * inner product Re(u^H v).  r: device float32 [nx][nk]; eta_out: device
 * complex64 [nx][nk]; must not alias.  The transposed interpolation is a
 * gather (no atomics): results are bitwise repeatable. */
int isam_adjoint(isam_plan_t p, const float* r, void* eta_out, void* stream);

/* Normal operator eta_out = A^H A eta with the residual pass fused: one
 * lateral transform pair instead of two.  Same layouts as above. */
int isam_normal(isam_plan_t p, const void* eta, void* eta_out, void* stream);

/* Step constant L >= ||A||^2 (replacing the fixed 1/N step of Alg. 1): power
 * iteration on A^H A for `iters` steps from a start vector x0 (device
 * complex64 [nx][nk], read only) or, if x0 is NULL, from a seeded
 * counter-based complex Gaussian (SplitMix64 + Box-Muller).  Norms are FP64.
 * *L_out = 1.01 * final Rayleigh quotient.  Synchronises the stream. */
int isam_lipschitz(isam_plan_t p, int iters, uint64_t seed, const void* x0, double* L_out,
                   void* stream);

/* lambda_max = max_i |(A^H y)_i| / w_i, the smallest lambda for which eta = 0
 * solves Eq. 12.  w may be NULL (w = 1).  Synchronises the stream. */
int isam_lambda_max(isam_plan_t p, const float* y, const float* w, double* out, void* stream);

/* Calibration gradient (Eq. 7 and 13 with the focal reference of the modulation c):
 * grad_out[0..2] = d/d(a2, a3, z_focus) of sum_{p,n} g[p][n] (A eta)[p][n], evaluated
 * at the plan's current calibration.  This is the calibration part of the
 * vector-Jacobian product of isam_forward with cotangent g (the object part is
 * isam_adjoint(g)).  With dc/dtheta = i D_theta c, D = ((k-k0)^2, (k-k0)^3, 2k - kz):
 *   grad_theta = -sum_{l,n} D_theta Im(conj(G[l][n]) c X[l][n]),  G = lateral DFT of g.
 * eta: device complex64 [nx][nk]; g: device float32 [nx][nk]; grad_out: host
 * double[3], in units of 1/(rad m^-2), 1/(rad m^-3) and 1/m of the three parameters.
 * Per-point terms are FP32, block sums FP32, the final sum FP64.  Synchronises the
 * stream.  Errors: EINVAL (NULL argument), ENONFINITE. */
int isam_calibration_grad(isam_plan_t p, const void* eta, const float* g, double* grad_out,
                          void* stream);

/* MBIR full-range ISAM by FISTA (Alg. 1) with step 1/L and threshold
 * lambda w_i / L (Eq. 14).  y: device float32 [nx][nk] measured spectra;
 * w: NULL or device float32 [nx][nk] (> 0); eta_out: device complex64
 * [nx][nk], receives z^k (plus (1/L) A^H(y - A z^k) if add_residual).
 * max_iter >= 0 iterations (0 returns the start point eta^1 = 0); tol > 0
 * enables the relative-residual stop of Eq. 15, evaluated on the device after
 * every update pass (the host reads the stop state every 16 iterations; the
 * iterations queued after the stopping one return at once, so eta_out is the
 * stopping iterate); tol = 0 runs exactly max_iter iterations with no host
 * synchronisation until the end.  L <= 0 runs
 * isam_lipschitz (50 steps, seed 0) first.  info may be NULL.  Synchronises
 * the stream at the end.  Errors: EINVAL, EALIAS, ENONFINITE (info->status). */
int isam_fista(isam_plan_t p, const float* y, float lambda, const float* w, int max_iter,
               float tol, double L, int add_residual, void* eta_out, isam_fista_info* info,
               void* stream);

/* Saved state of a FISTA solve (Alg. 1), for checkpoint and resume.  k: iterations done;
 * t: the momentum sequence value t^{k+1} the next iteration uses; data: caller-owned device
 * memory of isam_fista_state_bytes bytes holding the momentum point eta^{k+1} and the last
 * iterate z^k in the plan's internal layout (opaque; valid only for a plan of the same
 * geometry). */
typedef struct {
    int32_t k;
    double t;
    void* data;
} isam_fista_state;

/* Size in bytes of the device buffer of an isam_fista_state for plan p. */
int isam_fista_state_bytes(isam_plan_t p, int64_t* bytes);

/* isam_fista with checkpoint/resume and per-iteration records (Alg. 1, Eq. 15).
 * resume: NULL (start at eta^1 = z^0 = 0, t^1 = 1) or a state saved by an earlier call on a
 *   plan of the same geometry; iteration numbering continues at resume->k + 1, and running
 *   a then b iterations gives bit for bit what a + b iterations give.
 * save: NULL or a state whose data buffer receives the state after the last iteration run
 *   (the stopping iteration if Eq. 15 stopped the solve); save->k and save->t are set.
 *   save->data must not overlap y, w or eta_out; it may be resume->data.
 * history: NULL or host double[max_iter][3]; row i receives, for iteration i + 1 of this
 *   call, r_r of Eq. 15, ||A eta^k - y||^2 at the momentum point and sum_i w_i |z^k_i|
 *   (rows past info->iters_run are not written).  Forming them costs the Eq. 15 norms on
 *   every iteration.
 * Other arguments, results and errors as isam_fista; eta_out is unspecified when the
 * status is ENONFINITE. */
int isam_fista_ex(isam_plan_t p, const float* y, float lambda, const float* w, int max_iter,
                  float tol, double L, int add_residual, const isam_fista_state* resume,
                  isam_fista_state* save, double* history, void* eta_out, isam_fista_info* info,
                  void* stream);

/* The "direct IFFT" image of Eq. 9 (Sec. "Methods under test"), the reference the paper
 * compares MBIR with: each measured A-scan is dispersion-compensated by e^{-j phi(k)} and
 * transformed along k onto the full-range depth grid,
 *   eta_out[p][m + nk/2] = nk^{-1/2} sum_n y[p][n] e^{-j phi(k_n)} e^{-2 j k_n z_m},
 * with the operator's depth kernel (a plain inverse FFT over the sample index differs by a
 * unimodular phase per depth row and its scaling).  It holds half the object plus the
 * doubly dispersed conjugate mirror; A-scans are independent (no Stolt map, beam filter or
 * focus).  y: device float32 [nx][nk]; eta_out: device complex64 [nx][nk]; must not alias.
 * One nk-point LDS FFT per A-scan.  Errors: EINVAL (NULL), EALIAS. */
int isam_direct(isam_plan_t p, const float* y, void* eta_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): isam_direct without a plan.  The tables
 * the direct image needs (dispersion compensation, row phases, FFT twiddles) are built by a
 * kernel into a static device array of the library (100 KB, held by each GPU the library
 * runs on until the process ends); nothing is allocated.  g: geometry (nx, ny, nk,
 * lambda_c, dlambda, a2, a3 are read); y: device float32 [ny][nx][nk]; eta_out: device
 * complex64 [ny][nx][nk]; same result as isam_direct on a plan of g.  nk must be a power of
 * two from 16 to 4096 (the array's capacity): EUNSUPPORTED otherwise.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race and give wrong images; calls on one stream are ordered and safe.  Asynchronous.
 * Errors: EINVAL (NULL, bad optics), EUNSUPPORTED, EALIAS, ENODEV, EHIP. */
int isam_direct_static(const isam_geometry* g, const float* y, void* eta_out, void* stream);

/* Plan inspection (testing and diagnostics).  isam_plan_stolt writes, for lateral-frequency
 * column col (FFT order; col = lx * ny + ly for a volume) and every sample n < nk, the
 * oversampled grid position the NUFFT kernels use (Eq. 3 on the K = 2 nz grid): fl_out[n] =
 * floor(t), not reduced mod K, and tau_out[n] = t - floor(t); -1 for evanescent samples.
 * fl_out: device int32 [nk]; tau_out: device float32 [nk].  isam_plan_weights evaluates the
 * plan's min-max weight table (the interpolator the paper adopts, Sec. "Efficient and robust
 * ISAM through non-uniform FFT") as the kernels do, at tau (device float32 [n], in [0, 1)):
 * w_out (device complex64 [n][6]) receives u_1..u_6(tau), times the integer focal row's phase
 * e^{-2 pi i mi (tau + 3 - j) / K} that the plan folds into the table (none for z_focus = 0).
 * Both asynchronous.  Errors: EINVAL. */
int isam_plan_stolt(isam_plan_t p, int col, int32_t* fl_out, float* tau_out, void* stream);
int isam_plan_weights(isam_plan_t p, const float* tau, int n, void* w_out, void* stream);

/* Per-pass timing (profiling support).  enable = 1 clears the accumulators and
 * makes every later operator / FISTA call on the plan attach a HIP event pair
 * to each pass's kernel launch on its stream (the runtime stamps the pair with
 * that kernel's own begin and end); enable = 0 stops recording.  Elapsed
 * times are summed when a call completes (calls that synchronise) or here.
 * ms_out[ISAM_NPASS] and count_out[ISAM_NPASS] (either may be NULL) receive
 * the summed milliseconds and launch counts per pass:
 *   0 lateral FFT (forward)          1 Stolt NUFFT forward (in FISTA: with the data
 *   2 lateral C2R                      subtracted in lateral frequency)
 *   3 lateral R2C                    4 Stolt NUFFT adjoint
 *   5 lateral FFT (inverse)          6 FISTA update pass
 *   7 y transform of a volume (both directions; x passes count under 0, 2, 3, 5)
 *   8 direct image (isam_direct)
 * Synchronises the plan's last stream before reading. */
#define ISAM_NPASS 9
int isam_timing(isam_plan_t p, int enable, double* ms_out, int64_t* count_out);

/* ------------------------------------------------------------------------
 * Batches of B-scans of uneven size.
 *
 * A batch holds one plan per scan (each with its own geometry: nx, nk, optics
 * and calibration) and runs each pass of the operator (Eq. 5, 13, 16), its
 * adjoint (Eq. 17) and the FISTA iteration (Alg. 1) as one launch per group of
 * scans sharing a kernel specialisation (same nx for the lateral passes, same
 * nk for the NUFFT passes) instead of one launch per scan.  One FISTA
 * iteration is captured once in a hipGraph and replayed.  FISTA has a second
 * schedule, which runs each scan's own solve with the scans spread over the
 * batch's streams; the tuner picks one of the two.
 *
 * Packed buffers: scan i occupies elements [off[i], off[i+1]) of every packed
 * buffer (isam_batch_offsets), row-major [nx_i][nk_i] as for a single plan;
 * objects are complex64, spectra float32.  All data pointers are caller-owned
 * device memory; a batch may not run on two streams concurrently.
 * ------------------------------------------------------------------------ */
typedef struct isam_batch_s* isam_batch_t;

/* Flag of isam_batch_fista: launch the iteration's kernels one by one instead of
 * replaying the captured graph (same results, bit for bit; grouped schedule only). */
#define ISAM_BATCH_NO_GRAPH 1

/* FISTA schedules of a batch (isam_batch_set_schedule, isam_batch_tune):
 * GROUPED  one launch per pass per group of scans, the iteration replayed as a
 *          graph; every scan advances one iteration per replay (the default);
 * STREAMS  each scan's own solve (isam_fista on its plan) on one of four
 *          streams of the batch (each with a hardware queue of its own), scans
 *          dealt to streams by decreasing size, one host thread per stream
 *          enqueueing its scans' solves in turn, so that passes of different
 *          scans overlap.  Each scan's result is isam_fista's on its plan, bit for
 *          bit; the calling thread's device is used. */
#define ISAM_BATCH_SCHED_GROUPED 0
#define ISAM_BATCH_SCHED_STREAMS 1

/* Build a batch of nscans plans from geoms[0..nscans).  Errors: those of
 * isam_plan for any scan (the batch is then not created), EINVAL, ENOMEM. */
int isam_batch_plan(const isam_geometry* geoms, int nscans, void* stream, isam_batch_t* out);

/* offsets[0..nscans] (host int64): element offsets of the scans in packed buffers. */
int isam_batch_offsets(isam_batch_t b, int64_t* offsets);

/* The plan of scan i (owned by the batch; valid until isam_batch_destroy).  Its
 * single-scan calls use the same tables and tile widths as the batch; a
 * calibration set on it directly is picked up by the next batch call. */
int isam_batch_scan_plan(isam_batch_t b, int i, isam_plan_t* out);

/* isam_set_calibration for scan i, keeping the batch's records in step. */
int isam_batch_set_calibration(isam_batch_t b, int i, double a2, double a3, double z_focus,
                               void* stream);

/* Packed s = A eta per scan (isam_forward on every scan). */
int isam_batch_forward(isam_batch_t b, const void* eta, float* s_out, void* stream);

/* Packed eta = A^H r per scan (isam_adjoint on every scan). */
int isam_batch_adjoint(isam_batch_t b, const float* r, void* eta_out, void* stream);

/* FISTA on every scan (isam_fista per scan, all scans advancing together):
 * lambda: host float[nscans]; L: host double[nscans] or NULL (entries <= 0 are
 * computed by isam_lipschitz); w: packed weights or NULL; tol > 0 applies
 * Eq. 15 per scan on the device (a scan that has stopped keeps its iterate;
 * the loop ends when all have stopped or after max_iter iterations); info:
 * host isam_fista_info[nscans] or NULL; flags: 0 or ISAM_BATCH_NO_GRAPH.
 * Runs in the batch's schedule (ISAM_BATCH_SCHED_*).  Synchronises the stream.
 * Returns the first non-OK scan status, if any. */
int isam_batch_fista(isam_batch_t b, const float* y, const float* lambda, const float* w,
                     int max_iter, float tol, const double* L, int add_residual, int flags,
                     void* eta_out, isam_fista_info* info, void* stream);

/* Autotuner: for every group of scans with nx >= 192, times the batched update
 * pass (complex tiles) and R2C pass (real tiles) at tile widths 2, 4 and 8
 * lanes, `reps` launches each, and keeps the fastest; then times an 8-iteration
 * FISTA call on zero data in each schedule (one warm-up call, then `reps` calls,
 * host clock) and keeps the faster schedule.  Waits for earlier work on
 * `stream`, clobbers the scans' solver workspaces (not their tables), allocates
 * and frees two packed scratch buffers, and synchronises. */
int isam_batch_tune(isam_batch_t b, int reps, void* stream);

/* Set the FISTA schedule (ISAM_BATCH_SCHED_GROUPED or _STREAMS), e.g. from a
 * saved tuning; EINVAL for any other value. */
int isam_batch_set_schedule(isam_batch_t b, int sched);

/* The FISTA schedule in use. */
int isam_batch_schedule(isam_batch_t b, int* sched);

/* Tile widths in use: for up to cap lateral groups, nx and the lanes per tile of
 * the complex and real passes; *ngroups receives the number of groups. */
int isam_batch_tiles(isam_batch_t b, int32_t* nx, int32_t* sel_c, int32_t* sel_r, int32_t cap,
                     int32_t* ngroups);

/* Set the tile widths (lanes: 1, 2, 4 or 8) of the group with lateral length nx,
 * e.g. from a saved tuning.  Synchronises the device.  EINVAL if no group has
 * that nx. */
int isam_batch_set_tiles(isam_batch_t b, int32_t nx, int32_t sel_c, int32_t sel_r);

/* Release a batch and its plans (NULL is allowed). */
void isam_batch_destroy(isam_batch_t b);

/* Release a plan (NULL is allowed). */
void isam_destroy(isam_plan_t p);

/* Static, never-NULL description of an ISAM_* code. */
const char* isam_strerror(int code);

/* Sizes of a plan: nx, nk and the oversampled length K (any may be NULL). */
int isam_plan_dims(isam_plan_t p, int32_t* nx, int32_t* nk, int32_t* K);

#ifdef __cplusplus
}
#endif

#endif /* ISAM_H */
