/*
 * mipwa.h -- C ABI of libmipwa, an MI355X (gfx950) engine for the unbinned likelihood of a
 * model-independent partial-wave analysis (MIPWA) of D+ -> h- h+ h+.
 *
 * The method is that of "Model-independent partial wave analysis using a massively-parallel
 * fitting framework" (Sun, Aoude, dos Reis, Sokoloff):
 *   Sec. 2, Eq. 1  A(s12, s13) = sum_L sum_k c_k^L A_k^L(s12, s13), truncated at L = 2;
 *   Sec. 2         P/D waves: relativistic Breit-Wigner times a real spin-dependent angular factor;
 *   Sec. 2         S-wave: N boundary points s_k spanning the m^2(h+h-) spectrum, A_0(s_k) =
 *                  a_k exp(i phi_k) with a_k, phi_k free, and a cubic spline in the complex plane in
 *                  between (read as: natural spline of Re and Im through z_k = a_k exp(i phi_k));
 *   Sec. 4         Bose symmetrisation over the two h+h- axes: every amplitude is f(s12,s13)+f(s13,s12);
 *   Sec. 2, Sec. 4 unbinned maximum likelihood, with the normalisation integral recomputed from points
 *                  spread over the Dalitz plane in every iteration.
 * The quantity evaluated is
 *   -2 ln L = -2 sum_i ln|A(x_i)|^2 - 2 sum_i ln eps(x_i) + 2 n ln I,   I = sum_j w_j eps_j |A(x_j)|^2.
 *
 * Conventions
 *   Units: GeV, GeV^2, GeV^-1.  Particle 1 is the h-, particles 2 and 3 the identical h+ (m2 == m3).
 *   Parameter vector theta (P = 2N + 4R doubles, default polar S-wave form):
 *     [a_0, phi_0, ..., a_{N-1}, phi_{N-1},  |c_1|, arg c_1, ..., |c_R|, arg c_R,  m_1, G_1, ..., m_R, G_R]
 *   (mipwa_set_swave_form selects the Cartesian knot form or the isobar S-wave.)
 *   The S-wave is component 0 of Eq. 1 with coefficient 1.
 *   Every function returns an int status: MIPWA_OK (0) or a negative MIPWA_E_* code; no C++ exception
 *   crosses the ABI.  On error, mipwa_last_error(ctx) holds a message.
 *   A context is used by one thread at a time; separate contexts may be used from separate threads.
 *   Host input arrays are copied before a call returns; output arrays are allocated by the caller.
 */
#ifndef MIPWA_H
#define MIPWA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MIPWA_FP64 = 0, MIPWA_MIXED = 1 };

enum {
  MIPWA_OK = 0,
  MIPWA_E_INVAL = -1,      /* bad argument: sizes, masses, knots, points outside the Dalitz region */
  MIPWA_E_NOMEM = -2,      /* device or pinned host allocation failed, or a budget was exceeded */
  MIPWA_E_HIP = -3,        /* a HIP runtime call failed */
  MIPWA_E_STATE = -4,      /* call out of order (e.g. eval before events, params or norm points) */
  MIPWA_E_DOMAIN = -5,     /* non-finite -2 ln L (|A|^2 = 0 at an event); the value is +inf */
  MIPWA_E_NOCONV = -6,     /* the minimiser stopped without reaching the requested EDM */
  MIPWA_E_CANCELLED = -7,  /* a serving job was cancelled */
  MIPWA_E_BUSY = -8        /* a serving job has no result yet */
};

enum { MIPWA_MAX_KNOTS = 128, MIPWA_MAX_RES = 4 };

/* One P- or D-wave resonance (Sec. 2: spin-dependent relativistic Breit-Wigner).
 * spin in {0,1,2}; mass and width > 0; radius >= 0 is the Blatt-Weisskopf radius of the resonance.
 * The running width is Gamma(x) = width (q/q_r)^(2L+1) (mass/sqrt(x)) B_L(q,q_r)^2; barrier factors
 * B_L(q,q_r; radius) B_L(p,p_r; rD) with p the bachelor momentum in the resonance frame; Zemach
 * angular factors T_1, T_2. */
typedef struct {
  int spin;
  double mass;
  double width;
  double radius;
} mipwa_res;

/* Decay kinematics, D barrier radius rD >= 0, the N strictly increasing knot positions in m^2(h+h-)
 * (Sec. 2 boundary points; 2 <= N <= MIPWA_MAX_KNOTS; two knots give a straight-line S-wave, the
 * carrier of the isobar form below) and R <= MIPWA_MAX_RES resonances (spin 0 entries are the scalar
 * Breit-Wigners of an isobar S-wave). */
typedef struct {
  double M, m1, m2, m3, rD;
  int n_knots;
  const double* knots;
  int n_res;
  const mipwa_res* res;
} mipwa_model;

typedef struct mipwa_ctx mipwa_ctx;

/* Create a context on HIP device `device` computing in `precision` (MIPWA_FP64: all device arithmetic
 * in FP64; MIPWA_MIXED: FP32 point streams, amplitudes and spline, FP64 accumulation and host finish).
 * Errors: E_INVAL for an invalid model (m2 != m3, knots not increasing or out of range, spin outside
 * 0..2, width <= 0, radius < 0, a mass below its two-body threshold or above M - m3); E_HIP. */
int mipwa_create(const mipwa_model* model, int precision, int device, mipwa_ctx** out);
void mipwa_destroy(mipwa_ctx* ctx);
/* Message for the last failed call on ctx (never NULL; empty if none).  Valid until the next call. */
const char* mipwa_last_error(const mipwa_ctx* ctx);
const char* mipwa_strerror(int status);
/* Number of parameters P of the current S-wave form (2N + 4R, or 2 + 4R for the isobar form). */
int mipwa_n_params(const mipwa_ctx* ctx);

/* S-wave parameter form, which sets the layout of theta, the fixed mask and the gradient:
 *   MIPWA_SWAVE_POLAR (default): the knots as (a_k, phi_k), z_k = a_k e^{i phi_k} (Sec. 2);
 *   MIPWA_SWAVE_CARTESIAN: the knots as (Re z_k, Im z_k), the alternative the paper's abstract names
 *     in its source text; same model, the knot partials are dL/dRe z_k, dL/dIm z_k;
 *   MIPWA_SWAVE_ISOBAR: the S-wave of the isobar model (Sec. 2): one constant non-resonant term
 *     c_NR = |c_NR| e^{i arg c_NR}, entering A once, plus the model's spin-0 resonances as scalar
 *     Breit-Wigners; theta = [|c_NR|, arg c_NR, (|c_r|, arg c_r)_r, (m_r, Gamma_r)_r].  The model must
 *     have exactly two knots (they carry c_NR / 2 each).
 * Resets the parameters (set them again) and the fixed mask (masses and widths fixed).  Not available
 * in the serving API, whose jobs use the polar form.  Errors: E_INVAL (unknown form; isobar with
 * N != 2). */
enum { MIPWA_SWAVE_POLAR = 0, MIPWA_SWAVE_CARTESIAN = 1, MIPWA_SWAVE_ISOBAR = 2 };
int mipwa_set_swave_form(mipwa_ctx* ctx, int form);

/* How the normalisation integral I of Sec. 4 (recomputed at every evaluation) is formed:
 *   MIPWA_NORM_POINTS (default): a sweep over the normalisation points at every evaluation;
 *   MIPWA_NORM_QFORM: while every mass and width is fixed, A is linear in the spline polynomial
 *     coefficients of the two intervals of a point and in the c_r, so I is a sum over the occupied
 *     spline cells of v^T M_c conj(v) with per-cell moment matrices M_c of size (8 + R)^2, formed in
 *     one pass over the points whenever the resonance amplitudes are rebuilt.  Each evaluation then
 *     reads the moments instead of the points.  The same quantity up to rounding (an algebraic
 *     rearrangement, not a method of the paper); with a mass or width floated the point sweep is used.
 * Takes effect at the next evaluation.  Errors: E_INVAL (unknown mode). */
enum { MIPWA_NORM_POINTS = 0, MIPWA_NORM_QFORM = 1 };
int mipwa_set_norm_mode(mipwa_ctx* ctx, int mode);

/* Data events (the sample whose likelihood is maximised, Sec. 2).  s12[i], s13[i] are host arrays of n
 * doubles, each event inside the Dalitz region to within 1e-9 (M - m3)^2.  eff (nullable) gives the
 * efficiency at each event; it enters only the constant -2 sum ln eff.  If eff is NULL and an efficiency
 * table was set with mipwa_set_eff_table, the table is used; otherwise eff = 1.  Events are reordered
 * internally (the two h+h- coordinates of an event may be swapped: |A|^2 is symmetric, Sec. 4).
 * Replaces previously loaded events.  Errors: E_INVAL (n < 1, non-finite or outside values, eff <= 0). */
int mipwa_load_events(mipwa_ctx* ctx, const double* s12, const double* s13, const double* eff, int64_t n);

/* Normalisation points (Sec. 4: points over the Dalitz plane used to normalise the PDF each
 * iteration).  w[j] > 0 is the weight of point j (|D|/n for uniform phase-space points, the cell area for
 * a grid); eff as for mipwa_load_events.  I = sum_j w_j eff_j |A_j|^2.  Errors as mipwa_load_events. */
int mipwa_load_norm(mipwa_ctx* ctx, const double* s12, const double* s13, const double* w,
                    const double* eff, int64_t n);

/* Efficiency table: nx x ny float32 values at the bin centres of [lo, hi]^2 (row-major, index
 * [i12 * ny + i13]), read by bilinear interpolation between centres, constant beyond the outermost
 * centres.  Applied at the next mipwa_load_events / mipwa_load_norm whose eff argument is NULL.
 * Errors: E_INVAL (nx, ny < 2, hi <= lo, a value <= 0), E_HIP (allocation or upload); a failed call
 * leaves the previous table, or none, in force. */
int mipwa_set_eff_table(mipwa_ctx* ctx, const float* table, int nx, int ny, double lo, double hi);

/* Parameters held fixed (fixed[p] != 0) in mipwa_fit.  The same mask selects whether mass and width
 * partials are evaluated: when every mass and width is fixed (the default) the resonance amplitudes are
 * cached on the device and rebuilt only when a mass or width changes, and the mass/width entries of the
 * gradient are returned as 0; when any is floated the amplitudes and their mass/width derivatives are
 * computed on the fly in every evaluation.  Errors: E_INVAL (n != P). */
int mipwa_set_fixed(mipwa_ctx* ctx, const unsigned char* fixed, int n);

/* Set theta (P doubles, layout above).  Errors: E_INVAL (n != P, non-finite values, a width <= 0 or a
 * mass outside its kinematic range). */
int mipwa_set_params(mipwa_ctx* ctx, const double* theta, int n);

/* -2 ln L and its gradient at the current theta.  grad (nullable) receives P doubles.  Synchronous:
 * returns once the device has written the results to pinned host memory (the calling thread polls a
 * sequence word the finish kernel stores after them; the tail of that kernel may still be retiring on
 * the context's stream, which every call that replaces device buffers waits for).
 * Errors: E_STATE (no events, norm points or params), E_DOMAIN (non-finite value: *nll = +inf), E_HIP. */
int mipwa_eval(mipwa_ctx* ctx, double* nll, double* grad);

/* As mipwa_eval, asynchronously on `hip_stream` (a hipStream_t owned by the caller; NULL = the null
 * stream): d_out is a device pointer to 1 + P doubles that receives [-2 ln L, grad...] when the stream
 * reaches it.  The caller owns d_out and the stream.  No host synchronisation on the result; a
 * non-finite value is not reported as E_DOMAIN (inspect d_out). */
int mipwa_eval_async(mipwa_ctx* ctx, void* hip_stream, double* d_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the evaluation of mipwa_eval_async, with the same kernels, launch
 * shape and result, that allocates nothing.  Its scratch -- segment and job descriptors, resonance
 * constants, the per-block records and the group records -- lives in one static device array of 8 MiB
 * per GPU (held until the process ends) instead of context buffers; the events, normalisation points,
 * resonance cache and tables stay those the context allocated when the points were loaded.  At the
 * default launch shape (2 blocks per CU) every model up to 128 knots and 4 resonances fits.
 * Every call on one GPU shares that array and it keeps the last call's contents: calls that overlap on
 * one GPU (from any context, on streams not ordered with each other) race.  Calls on one context are
 * ordered with its other evaluations like mipwa_eval_async.  d_out: device pointer to 1 + P doubles.
 * Errors: E_INVAL (d_out NULL; a launch shape whose records exceed the array, see mipwa_set_launch),
 * E_STATE (nothing loaded, no parameters, or the quadratic-form normalisation, whose per-cell moments
 * are context memory: use MIPWA_NORM_POINTS), E_HIP. */
int mipwa_eval_noalloc(mipwa_ctx* ctx, void* hip_stream, double* d_out);

/* Component integrals over the normalisation points (Sec. 2, Eq. 1 components; component 0 = S-wave,
 * r = 1..R the resonances at the current theta): I_jk = sum_p w_p [eff_p] A_j A_k^*, K = R + 1.
 * with_eff = 0 omits the efficiency (for fit fractions).  Ijk receives 2 K K doubles (re, im), row-major. */
int mipwa_integrals(mipwa_ctx* ctx, int with_eff, double* Ijk);

/* Fit fractions FF_jk = Re(c_j c_k^* I_jk) / sum_jk c_j c_k^* I_jk at the current theta, with I
 * computed without efficiency; ff receives K K doubles.  */
int mipwa_fit_fractions(mipwa_ctx* ctx, double* ff);

/* Maximum-likelihood fit (Sec. 2: {a_k, phi_k} and the c's determined by an unbinned ML fit; Sec. 4:
 * normalisation recomputed every iteration).  Quasi-Newton BFGS with a strong-Wolfe line search over the
 * parameters not marked fixed (mipwa_set_fixed), from theta_inout; stops when the estimated distance to
 * the minimum EDM = g^T B g / 2 (B the inverse-Hessian estimate) falls below tol_edm.  Then H is taken by
 * central differences of the analytic gradient, cov = 2 H^-1 over the floated parameters (zero rows for
 * fixed ones), and each (magnitude, phase) pair is folded to magnitude >= 0, phase in (-pi, pi].
 * cov_out (nullable) receives P*P doubles.  Errors: E_NOCONV (max_iter reached; results still
 * written), E_STATE, E_DOMAIN (start point non-finite). */
typedef struct {
  double tol_edm;   /* default 1e-6 if <= 0 */
  int max_iter;     /* default 1000 if <= 0 */
  int hessian;      /* 1: finite-difference Hessian and covariance at the end; 0: skip (cov from B) */
} mipwa_fit_opts;
typedef struct {
  double nll, edm;
  int n_iter, n_eval, status;
} mipwa_fit_info;
int mipwa_fit(mipwa_ctx* ctx, const mipwa_fit_opts* opts, double* theta_inout, double* cov_out,
              mipwa_fit_info* info);

/* Toy Monte Carlo (Sec. 4: samples generated from the Dalitz-plot PDF) by accept-reject on
 * f = |A|^2 eff at theta, on the device.  Candidate i uses Philox4x32-10 (Salmon et al., SC'11) with
 * counter (i mod 2^32, i div 2^32, stream, 0) and key (seed mod 2^32, seed div 2^32): stream 0 gives
 * (u12, u13), stream 1 gives v, each double from two words as ((a>>5) 2^26 + (b>>6)) 2^-53; the
 * candidate is s = smin + (smax - smin) u, kept if inside the Dalitz region and f > v fmax.  The first n
 * accepted candidates in candidate order are written to the host arrays s12_out, s13_out.  The
 * efficiency is the table of mipwa_set_eff_table if set, else 1.  *exceeded (nullable) is set to 1 if
 * any examined candidate had f > fmax (the sample is then not exact: raise fmax and repeat);
 * *n_candidates (nullable) receives the number of candidates examined.  Does not change the context's
 * loaded points.  Errors: E_INVAL (n < 1, fmax <= 0, wrong theta length). */
int mipwa_generate(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, double fmax,
                   int64_t n, double* s12_out, double* s13_out, int* exceeded, int64_t* n_candidates);

/* Largest f = |A|^2 eff over the first n_probe candidates inside the Dalitz region of key `seed`
 * (same candidate stream as mipwa_generate). */
int mipwa_density_max(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, int64_t n_probe,
                      double* fmax_out);

/* The whole toy procedure (Sec. 4: toy samples generated from the Dalitz-plot PDF; the bound rule is
 * this library's reading, the paper states none): fmax = 1.5 x mipwa_density_max over n_probe
 * inside-candidates of key seed + 1000, then mipwa_generate with key `seed`; while any examined
 * candidate exceeds fmax, fmax is doubled and the sample drawn again from the first candidate.  Writes
 * n points to the host arrays s12_out, s13_out and the final bound to *fmax_out (nullable).  Errors:
 * as mipwa_generate, and E_INVAL for n_probe < 1 or a zero density over the probe. */
int mipwa_toy(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, int64_t n_probe, int64_t n,
              double* s12_out, double* s13_out, double* fmax_out);

/* Device times of the most recent timed evaluations (see mipwa_set_timing), in milliseconds: *total_ms
 * from before the first launch to the end of the finish, *stream_ms of the streaming likelihood kernel
 * alone; a figure that the last two timed evaluations did not record is NaN.  Nullable outputs.
 * Errors: E_STATE (nothing timed yet). */
int mipwa_last_timing(const mipwa_ctx* ctx, double* total_ms, double* stream_ms);

/* Device timing from HIP events recorded on the evaluation's stream (synchronous and asynchronous
 * evaluations).  period 0 turns it off; period n >= 1 times every n-th evaluation, and the timed
 * evaluations alternately record the whole evaluation (before the first launch to after the finish)
 * and the streaming kernel alone: each recorded event adds device time to its evaluation (a few
 * microseconds), so a sample every few evaluations leaves the rate of the others as it is.  Resets
 * the statistics.  mipwa_timing_stats returns the number of timed evaluations, the mean time of the
 * whole evaluation and the mean time of the streaming kernel over the evaluations that recorded each,
 * in milliseconds (NaN when none did).  Errors: E_INVAL (period < 0). */
int mipwa_set_timing(mipwa_ctx* ctx, int period);
int mipwa_timing_stats(const mipwa_ctx* ctx, int64_t* count, double* mean_total_ms, double* mean_stream_ms);

/* Measured streaming-read ceiling of a GPU, the denominator beside the datasheet peak when the
 * likelihood sweep's bandwidth is reported: a buffer of `bytes` (>= 1 MiB) is read with 16-byte
 * non-temporal loads and no other work, `reps` times for each of four grid sizes (4 to 32 blocks of 256
 * threads per CU) after one warm-up; *gbs receives the best rate in GB/s.  Allocates and frees its own
 * buffer.  Errors: E_INVAL, E_NOMEM, E_HIP. */
int mipwa_read_bandwidth(int device, int64_t bytes, int reps, double* gbs);

/* Launch shape of the streaming kernel: blocks (0 = default) and waves per block (0 = default, 1..16).
 * Takes effect at the next load.  Errors: E_INVAL. */
int mipwa_set_launch(mipwa_ctx* ctx, int blocks, int waves_per_block);

/* ---- toy-fit serving with continuous batching -------------------------------------------------
 * A server fits many independent toy samples (Sec. 4: fits of toy samples generated from the
 * Dalitz-plot PDF) against one shared normalisation sample.  Jobs wait until their device footprint
 * fits the HBM budget, then load (cell sort and resonance cache, a few loads at a time, first come
 * first served) and run the BFGS fit of mipwa_fit in a worker thread; a job's result is available
 * before its device memory has gone back to the server's pool.  Every evaluation a job needs is batched with the pending
 * evaluations of other active jobs into a single launch of the streaming kernel.  Up to two steps are
 * in flight: while one runs, the next is formed from the jobs outside it and queued behind it, so the
 * jobs' host work overlaps the device's (a step formed with none in flight takes at most half of the
 * active jobs, which splits them into two groups that alternate).  A step is launched once every
 * active job outside the steps in flight has asked, or 50 us after its first request; jobs admitted
 * while a step runs join a later one.  A job's result does not depend on which other jobs share its steps (its
 * kernel blocks and reduction order depend only on its own sizes).  Serving jobs keep masses and
 * widths fixed.  The server is thread-safe.  With MIPWA_SERVE_TRACE set in the environment, admission,
 * loading, completion and the scheduler's time split are printed to stderr. */
typedef struct mipwa_server mipwa_server;
typedef struct {
  double fits_per_s;   /* finished jobs / (last completion - first submission) */
  double p50_s, p99_s; /* time-to-fit percentiles (submission to completion) */
  int64_t n_done, n_active, n_queued;
  int64_t peak_bytes;  /* largest admitted device footprint (events, scratch, normalisation sets) */
  int64_t steps;       /* batched launches so far */
  double mean_batch;   /* mean number of jobs per launch */
  double step_device_s; /* mean device time of a step (HIP events around every 17th step's kernels) */
  double device_busy;  /* step_device_s x steps / (last completion - first submission) */
} mipwa_serve_stats;

/* Create a server on `device` in `precision`; hbm_budget_bytes = 0 uses 80% of the free memory.
 * Errors: E_INVAL, E_HIP. */
int mipwa_server_create(int device, int precision, size_t hbm_budget_bytes, mipwa_server** out);
/* The shared normalisation sample (host arrays copied; weights as in mipwa_load_norm).  Must be set
 * before the first submission and cannot be replaced once a job has used it (E_STATE). */
int mipwa_server_set_norm(mipwa_server* s, const double* s12, const double* s13, const double* w, int64_t n);
/* Queue one fit: model, n events (host arrays, copied), start theta0 (P doubles), fixed mask (P bytes,
 * nullable: the first resonance coefficient and every mass and width fixed), options (nullable:
 * tol_edm 1e-4, max_iter 1000, no Hessian).  The masses and widths stay at theta0's values; jobs with
 * the same knots and the same masses and widths share one set of normalisation moments (formed by the
 * first of them to load, the same numbers whichever does).  *job_id receives the job's id.  Errors:
 * E_INVAL (model, theta0, a floated mass or width), E_STATE (no normalisation sample), E_NOMEM (the job
 * alone exceeds the budget). */
int mipwa_server_submit(mipwa_server* s, const mipwa_model* model, const double* s12, const double* s13, int64_t n,
                        const double* theta0, const unsigned char* fixed, const mipwa_fit_opts* opts,
                        int64_t* job_id);
/* As mipwa_server_submit, without copying the events: the server reads s12 and s13 (host memory, not
 * pinned) when the job is admitted and loaded, so the caller keeps both arrays valid and unchanged
 * until mipwa_server_poll or mipwa_server_wait has returned the job's final status (or the server is
 * destroyed).  Submitting many large jobs at once then costs no host copy in the caller's thread. */
int mipwa_server_submit_borrowed(mipwa_server* s, const mipwa_model* model, const double* s12, const double* s13,
                                 int64_t n, const double* theta0, const unsigned char* fixed,
                                 const mipwa_fit_opts* opts, int64_t* job_id);
/* Result of a job: MIPWA_E_BUSY while queued or running, MIPWA_E_CANCELLED, otherwise the fit status
 * (MIPWA_OK or MIPWA_E_NOCONV) with theta_out (P doubles, nullable), info (nullable) and the
 * time-to-fit in seconds (nullable) filled in; another negative code if loading or fitting failed. */
int mipwa_server_poll(mipwa_server* s, int64_t job_id, double* theta_out, mipwa_fit_info* info, double* latency_s);
/* As mipwa_server_poll, blocking until the job finishes or timeout_s (> 0) elapses. */
int mipwa_server_wait(mipwa_server* s, int64_t job_id, double timeout_s, double* theta_out, mipwa_fit_info* info,
                      double* latency_s);
/* Cancel a queued or running job (it stops at its next evaluation); other jobs are unaffected. */
int mipwa_server_cancel(mipwa_server* s, int64_t job_id);
int mipwa_server_stats(mipwa_server* s, mipwa_serve_stats* stats);
/* The message of the server's most recent error, from any thread (a failed call, or a failed batched
 * step: the jobs that step carried end with its status and message).  The string belongs to the
 * calling thread and stays valid until that thread's next call of this function. */
const char* mipwa_server_last_error(const mipwa_server* s);
/* Cancel every job, join the worker threads and free the device memory. */
void mipwa_server_destroy(mipwa_server* s);

#ifdef __cplusplus
}
#endif

#endif /* MIPWA_H */
