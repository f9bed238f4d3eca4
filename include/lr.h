/*
 * lr.h -- C ABI of the MI355X low-rank Lindblad readout integrator.
 *
 * What is computed (the paper's supplement S1.A, eq. "lowrank_diagonal" and
 * eq. "nosse"): the density matrix is kept as rho = B B^ with B an N x M
 * complex factor, and B follows
 *
 *     dB/dt = -i H(t) B + O[B],
 *     O[B]  = 1/2 sum_k [ L_k B (B^+ L_k B)^  -  L_k^ L_k B ],   B^+ = (B^B)^-1 B^
 *
 * for the transmon-resonator-filter readout model (main text, Hamiltonian
 * eq. "hamiltonianpurcell", master equation eq. "hamiltonian") in the form
 *
 *     H(t) = w_q n_q + alpha/2 n_q(n_q-1) + w_r n_r + w_f n_f
 *            + g (b+b^)(a+a^) + G (a+a^)(f+f^) + d(t) (f+f^),
 *     L_1 = sqrt(kappa_f) f,   L_2 = sqrt(gamma_1) b,
 *
 * integrated by classic fixed-step RK4.  Each right-hand side evaluation
 * applies H_eff = H - i/2 sum_k L_k^ L_k and L_k mode-wise, forms the Gram
 * G = B^ B and C_k = B^ L_k B, solves G X_k = C_k in FP64 and assembles
 * dB/dt = -i H_eff B + 1/2 sum_k (L_k B) X_k^.  The integrators solve by
 * Gauss-Jordan elimination of the augmented [G | C_1 C_2] without pivoting
 * (its pivots are those of G = L D L^, positive iff G is positive definite);
 * the multi-kernel path behind lr_rhs factors G by Cholesky.
 *
 * Units: rad/ns and ns.  Basis index n = (i_q d_r + i_r) d_f + i_f.
 *
 * Memory and ownership.  B is passed as device memory, column-major N x M,
 * interleaved complex FP64 (lr_c64): element (n, j) at d_B[n + N*j].  The
 * caller owns every device buffer (B, dB, observation records, workspace);
 * the library owns only host-side descriptors created by lr_init and freed
 * by lr_destroy, and never frees caller memory.  All calls that take device
 * pointers enqueue work on the stream given to lr_bind and return without
 * waiting; errors found on the device (non-positive Gram pivot, non-finite
 * state) are reported by lr_status, which synchronises the stream.
 * Argument errors are reported synchronously by the return code and nothing
 * is enqueued.  No call throws across the ABI.
 */
#ifndef LR_H
#define LR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } lr_c64;

/* Model parameters (rad/ns).  d_q >= 2 (g and e must exist), d_r, d_f >= 1.
 * kind LR_MODEL_DUFFING (0): the Duffing transmon w_q n + alpha/2 n (n - 1)
 *   and the couplings g (b+b^)(a+a^), G (a+a^)(f+f^); drive d(t) (f + f^).
 * kind LR_MODEL_TRANSMON (1): the paper's Hamiltonian (main text, eq.
 *   "hamiltonianpurcell") in the bare resonator/filter basis with the
 *   transmon in its eigenbasis (supplement S2.A): levels E_t[0..d_q-1], charge
 *   operator n_t (d_q x d_q, row-major, real symmetric), couplings
 *   i g n_t (a^ - a) and -G (a^ - a)(f^ - f) (G is the paper's J), drive
 *   d(t) i (f^ - f); w_q and alpha unused; d_q <= LR_MAX_DQ.  In the drive
 *   frame the rotation counts the transmon level index as its excitation
 *   number (levels E_q - w_d q), every term kept.  This kind runs in the
 *   packed batch schedule only (fixed RK4 or adaptive steps; LR_ERR_ARG
 *   elsewhere).
 * kind LR_MODEL_NORMAL (2): the same Hamiltonian in the resonator-filter
 *   normal-mode basis (supplement S2.D; S2.E, eq. "hamiltonian_rotated"):
 *   the d_r slot holds the lower mode c_l (frequency w_r), the d_f slot the
 *   upper mode c_u (frequency w_f), and S[0..3], S[4..7] are the rows of the
 *   transformation a = S[0] c_u^ + S[1] c_l^ + S[2] c_l + S[3] c_u and
 *   f = S[4] c_u^ + S[5] c_l^ + S[6] c_l + S[7] c_u.  H = E_q + w_l n_l +
 *   w_u n_u + i g n_t (mu_l (c_l^ - c_l) + mu_u (c_u^ - c_u)) + d(t) i (nu_l
 *   (c_l^ - c_l) + nu_u (c_u^ - c_u)) with mu_l = S[2] - S[1], mu_u = S[3] -
 *   S[0], nu_l = S[6] - S[5], nu_u = S[7] - S[4] (G unused).  The filter jump
 *   L_1 = sqrt(kappa_f) f moves the state across resonator layers and raises
 *   as well as lowers; -1/2 L_1^ L_1 is applied as the product of the
 *   truncated operators.  In the drive frame every creation term of f carries
 *   e^{i w_d t} and every annihilation term e^{-i w_d t}.  Packed batches
 *   only, fixed RK4 or adaptive steps (LR_ERR_ARG elsewhere), FP64,
 *   d_q <= LR_MAX_DQ.  Its records hold <c_l> in the <a> columns and the
 *   filter field <f> (f as above, the field of the readout separation) in the
 *   <f> columns; in the drive frame <f> is e^{i w_d t} times its lab-frame
 *   value, as for the other kinds, t the record's time.
 * Kinds 0 and 1: L_1 = sqrt(kappa_f) f; every kind: L_2 = sqrt(gamma_1) b, b
 * the ladder sum_n sqrt(n) |n-1><n| of the transmon levels. */
#define LR_MODEL_DUFFING 0
#define LR_MODEL_TRANSMON 1
#define LR_MODEL_NORMAL 2
#define LR_MAX_DQ 8
typedef struct {
  int32_t d_q, d_r, d_f;
  int32_t kind;                   /* LR_MODEL_DUFFING, LR_MODEL_TRANSMON or LR_MODEL_NORMAL */
  double  w_q, alpha, w_r, w_f;   /* Duffing transmon w_q n + alpha/2 n(n-1); bare modes */
  double  g, G;                   /* g (b+b^)(a+a^),  G (a+a^)(f+f^)  (kind 0)           */
  double  kappa_f, gamma_1;       /* L_1 = sqrt(kappa_f) f,  L_2 = sqrt(gamma_1) b      */
  double  E_t[LR_MAX_DQ];         /* kinds 1, 2: transmon levels                        */
  double  n_t[LR_MAX_DQ * LR_MAX_DQ];  /* kinds 1, 2: charge operator, row-major d_q x d_q */
  double  S[8];                   /* kind 2: rows of a and f over (c_u^, c_l^, c_l, c_u)  */
} lr_model_t;

/* Drive coefficient d(t) multiplying (f + f^).
 *   LR_PULSE_FLATTOP:    d(t) = amp w(t) cos(w_d t)
 *   LR_PULSE_PIECEWISE6: d(t) = sum_{s=1,2} A_s w_s(t) cos((w_d + Delta_s) t + phi_s),
 *                        p = {A_1, phi_1, Delta_1, A_2, phi_2, Delta_2}
 * w(t) = r(t) r(T-t) with r(x) = 0 (x<0), (1-cos(pi x/t_ramp))/2 (0<=x<t_ramp), 1 else;
 * w_1 = r(t)(1-c(t)), w_2 = r(T-t) c(t), c a cosine cross-fade of length t_ramp
 * centred at T/2.  Every amplitude must satisfy |A| < 2 pi 0.4 rad/ns (the
 * drive bound of supplement S3.B-C), else LR_ERR_PULSE. */
enum { LR_PULSE_FLATTOP = 0, LR_PULSE_PIECEWISE6 = 1, LR_PULSE_STEPWISE = 2 };
/* LR_PULSE_STEPWISE (supplement S2.C, smoothed stepwise function): the complex
 * envelope Omega(t) = sum_{j=1}^{n} (h_{j+1} - h_j) / (1 + e^{-(t - j T / n) / sigma})
 * with n = nh + 1 logistic steps, h_1 = h_{n+1} = 0 (the drive is off before the
 * first and after the last step) and the nh complex heights h_2 .. h_n in
 * h[2 k], h[2 k + 1] (re, im), on the carrier: d(t) = Re[Omega(t) e^{-i w_d t}].
 * Requires 1 <= nh <= LR_PULSE_MAX_H, sigma > 0, T > 0 and every |h_k| below the
 * drive bound. */
#define LR_PULSE_MAX_H 63
/* frame: the frame the state B is integrated in (and reported in).
 *   LR_FRAME_LAB    the lab frame.
 *   LR_FRAME_DRIVE  the frame rotating at the carrier w_d (supplement S2.E,
 *                   eq. "hamiltonian_rotated", with every counter-rotating
 *                   term kept): B' = U B with U = exp(i w_d t (n_q + n_r + n_f)),
 *                   H' = U H U^ - w_d (n_q + n_r + n_f), i.e. mode frequencies
 *                   w - w_d, coupling pairs b^a^, a^f^ times e^{2 i w_d t}
 *                   (b a, a f times the conjugate) and the drive d(t) on
 *                   f^ e^{i w_d t} + f e^{-i w_d t}.  The dissipator is
 *                   unchanged.  Observation records hold the rotating-frame
 *                   <a>' = e^{i w_d t}<a> and <f>' = e^{i w_d t}<f>;
 *                   populations, traces and the readout loss are frame-free.
 * Any other value is LR_ERR_PULSE. */
enum { LR_FRAME_LAB = 0, LR_FRAME_DRIVE = 1 };
typedef struct {
  int32_t kind;
  int32_t frame;
  double  w_d, amp, t_ramp, T;
  double  p[6];
  int32_t nh;                          /* LR_PULSE_STEPWISE: number of heights */
  int32_t reserved;
  double  sigma;                       /* LR_PULSE_STEPWISE: logistic steepness (ns) */
  double  h[2 * LR_PULSE_MAX_H];       /* LR_PULSE_STEPWISE: heights h_2 .. h_n */
} lr_pulse_t;

/* Arithmetic of the operator applications (H_eff and L_k on B), the jump
 * assembly and the Gram / cross products of lr_integrate and lr_batch_run:
 *   LR_FP64    FP64 throughout;
 *   LR_FP32    operands rounded to FP32, FP32 products and accumulation;
 *   LR_BF16X3  operands rounded to FP32 and split into BF16 parts, each
 *              product formed from the three leading part products with FP32
 *              accumulation (evaluated on the vector ALU).
 * The M x M solve, the reduction of the Gram partials across the state and
 * the RK4 accumulation of B are FP64 in every mode.  lr_rhs and
 * lr_observables always evaluate in FP64; the reduced modes need the
 * persistent on-chip integrator (LR_ERR_ARG from lr_integrate otherwise).
 * In the packed batch schedule the modes apply to the Gram and cross
 * products only, which run on the matrix cores (LR_BATCH_PACKED_MFMA64). */
enum { LR_FP64 = 0, LR_FP32 = 1, LR_BF16X3 = 2 };

enum {
  LR_OK = 0,
  LR_ERR_ARG = -1,          /* invalid argument (dims, M, sizes, null pointers)   */
  LR_ERR_OOM = -2,          /* workspace smaller than lr_workspace_bytes          */
  LR_ERR_HIP = -3,          /* a HIP runtime call failed                          */
  LR_ERR_GRAM_NOT_PD = -4,  /* a pivot of B^B (LDL^ / Cholesky) <= 0 (device, via lr_status) */
  LR_ERR_NONFINITE = -5,    /* non-finite B or Gram (device, via lr_status)       */
  LR_ERR_PULSE = -6,        /* drive amplitude above the bound, or bad kind       */
  LR_ERR_STATE = -7,        /* call order (e.g. no workspace bound)               */
  LR_ERR_TIMEOUT = -8,      /* a bounded device-side wait expired (via lr_status) */
  LR_ERR_STEP = -9          /* adaptive step size underflow or step budget spent (via status) */
};

typedef struct lr_ctx lr_ctx_t;

/* Create a context for one trajectory shape.  Rejects dims < 1, d_q < 2,
 * M < 1, M > N, M > LR_MAX_M, unknown precision.  Host allocation only. */
#define LR_MAX_M 32
int lr_init(lr_ctx_t** ctx, const lr_model_t* model, int32_t M, int32_t precision);

/* Exact device workspace size in bytes for this context (256-byte aligned
 * start required).  Used for admission by HBM footprint. */
size_t lr_workspace_bytes(const lr_ctx_t* ctx);

/* Attach caller-owned device workspace (>= lr_workspace_bytes) and a HIP
 * stream (hipStream_t, may be NULL for the default stream). */
int lr_bind(lr_ctx_t* ctx, void* d_workspace, size_t bytes, void* stream);

/* One right-hand side evaluation dB = f(t, B) (supplement S1.A, eq. "nosse").
 * d_B and d_dB: device, column-major N x M lr_c64; they must not overlap. */
int lr_rhs(lr_ctx_t* ctx, const lr_pulse_t* pulse, double t, const lr_c64* d_B, lr_c64* d_dB);

/* Classic RK4 from B(t0) over nsteps steps of dt (step n starts at t0 + n dt).
 * d_B: device, in B(t0), out B(t0 + nsteps dt).  If obs_stride > 0, d_obs
 * (device, double) receives (nsteps / obs_stride + 1) records of
 * LR_OBS_LEN(d_q) doubles: at step 0 and after every obs_stride-th step.
 * Rejects dt <= 0, nsteps < 0, obs_stride < 0, a bad pulse. */
int lr_integrate(lr_ctx_t* ctx, const lr_pulse_t* pulse, double t0, double dt, int64_t nsteps,
                 lr_c64* d_B, int32_t obs_stride, double* d_obs);

/* Observation record of B (device) into d_out (device, LR_OBS_LEN(d_q) doubles):
 *   [Re<a>, Im<a>, Re<f>, Im<f>, tr rho, tr rho^2, P_q(0), ..., P_q(d_q-1)]
 * with <O> = tr(O rho) unnormalised (main text beta = tr(rho f); populations of
 * supplement eq. "transmon_ionization"), tr rho^2 = ||B^B||_F^2. */
#define LR_OBS_LEN(d_q) (6 + (d_q))
int lr_observables(lr_ctx_t* ctx, const lr_c64* d_B, double* d_out);

/* Spectrum of the low-rank density matrix (supplement S1.B, "Validity"):
 * the eigenvalues p_1 >= ... >= p_M of G = B^B, which are the nonzero
 * eigenvalues of rho = B B^ (the weights p_j of eq. "lowrank_diagonal").
 * p_M / p_1 is the paper's control quantity of the approximation and
 * sum_j p_j^2 = tr rho^2 its purity.  d_B: device, N x M in the layout of
 * lr_integrate; d_eval: device, M doubles, written in descending order.
 * FP64 throughout (Jacobi rotations of the real 2M x 2M form of G), one
 * workgroup, asynchronous on the bound stream.  Each p_j is accurate to
 * about 1e-15 ||G||_2 in absolute terms. */
int lr_spectrum(lr_ctx_t* ctx, const lr_c64* d_B, double* d_eval);

/* Synchronise the bound stream and return the first device-side error of the
 * last lr_integrate / lr_rhs / lr_observables (LR_OK if none); *failed_step
 * (may be NULL) receives the RK step index at which it occurred. */
int lr_status(lr_ctx_t* ctx, int64_t* failed_step);

/* Kernel timing telemetry.  While enabled, every launch of the integrator's
 * main kernel made by lr_integrate -- a chunk of steps of the persistent
 * on-chip kernel, or one stage of the multi-kernel fallback -- and of the
 * fallback's Gram solve kernel is bracketed by HIP events on the bound
 * stream (up to the first LR_PROFILE_MAX launches of each after enabling;
 * enabling again resets the counters).  lr_profile_read synchronises the
 * stream and returns the summed kernel times (ms) and launch counts. */
#define LR_PROFILE_MAX 4096
int lr_profile_enable(lr_ctx_t* ctx, int32_t on);
/* Bounded waits of the on-chip integrator's group barriers (failure
 * handling).  Every wait of a workgroup for the others polls at most `spins`
 * times (0: the default, 2^20 polls, far above any healthy wait) before it
 * gives up, ends its trajectory's whole workgroup group and reports
 * LR_ERR_TIMEOUT through lr_status; the context stays usable.  never != 0
 * makes every barrier wait for a value that no workgroup writes, so that each
 * wait expires after `spins` polls: a deterministic way for tests to drive the
 * timeout path from the host.  Applies to later lr_integrate calls. */
int lr_wait_limits(lr_ctx_t* ctx, uint32_t spins, int32_t never);
int lr_profile_read(lr_ctx_t* ctx, double* stage_ms, int64_t* stage_launches, double* solve_ms,
                    int64_t* solve_launches);

/* Readout figures of merit of a g/e pair from their observation series
 * (Supplement S3.A eqs. "SNR", "separation_error", "assignment_error"; S3.B
 * eqs. "transmon_ionization", "loss_function"):
 *   SNR       = sqrt(2 eta kappa_f int_0^tau |<f>_e - <f>_g|^2 dt)
 *   eps_sep   = erfc(SNR / 2) / 2,   eps_decay = tau gamma_1 / 2,   eps_a = eps_sep + eps_decay
 *   T         = (1 / tau) sum_{g,e} sum_{k = 2}^{d_q - 1} int_0^tau P_q(k) dt
 *   Lambda    = log10(eps_a + T)
 * d_obs_g, d_obs_e: device, nsamples (>= 2) records of LR_OBS_LEN(d_q)
 * doubles as written by lr_integrate, sampled every h ns (tau = h
 * (nsamples - 1)); integrals are composite trapezoids on that grid.
 * d_out: device, 6 doubles {SNR, eps_sep, eps_decay, eps_a, T, Lambda}.
 * Enqueued on `stream` (NULL: the null stream); LR_ERR_ARG for invalid
 * arguments. */
int lr_readout_loss(const double* d_obs_g, const double* d_obs_e, int64_t nsamples, int32_t d_q, double h,
                    double kappa_f, double gamma_1, double eta, double* d_out, void* stream);

/* Dense full-Lindblad comparison solve (Supplement S1.A, eq.
 * "master_equation" with the dissipator of eq. "lindblad_dissipator"): the
 * same model, drive and classic RK4 stage times as lr_integrate, on the full
 * N x N density matrix instead of the low-rank factor.
 * d_rho: device, row-major N x N interleaved complex FP64 in the basis order
 * of B (n = (q d_r + r) d_f + f), Hermitian; in rho(t0), out rho(t0 + nsteps
 * dt).  d_workspace: device, >= lr_dense_workspace_bytes(m) bytes (4 N^2
 * complex), owned by the caller.  obs_stride / d_obs: records as in
 * lr_integrate, computed from rho.  Enqueued on `stream`; N <= 16384.
 * Returns LR_ERR_ARG / LR_ERR_PULSE for invalid arguments. */
size_t lr_dense_workspace_bytes(const lr_model_t* m);
int lr_dense_integrate(const lr_model_t* m, const lr_pulse_t* pulse, double t0, double dt, int64_t nsteps,
                       lr_c64* d_rho, int32_t obs_stride, double* d_obs, void* d_workspace, size_t bytes,
                       void* stream);

/* Operator application on its own (supplement S1.A: the H_eff B term of the
 * right-hand side of eq. "nosse"): Z = H_eff(t) B, with H_eff = H(t) -
 * i/2 (kappa_f n_f + gamma_1 n_q) the model's non-Hermitian Hamiltonian
 * (kind LR_MODEL_DUFFING) in the lab frame or, with pulse->frame =
 * LR_FRAME_DRIVE, in the frame rotating at the carrier as lr_integrate takes
 * it.  d_B, d_Z: device, column-major N x ncols interleaved complex FP64
 * (column j at d_B + N j); columns are independent, so the factors of many
 * trajectories of one model at one time may lie side by side (ncols = K M).
 * B and Z must not overlap.  The integrators fuse this operation into their
 * stage kernels; this streaming pass reads B once and writes Z once.
 * Enqueued on `stream` (NULL: the null stream).  LR_ERR_ARG for invalid
 * arguments, N > 8192 or another model kind; LR_ERR_PULSE for a bad pulse. */
int lr_apply_heff(const lr_model_t* model, const lr_pulse_t* pulse, double t, const lr_c64* d_B, int64_t ncols,
                  lr_c64* d_Z, void* stream);

/* lr_integrate for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * integration -- the persistent on-chip path of lr_init + lr_bind +
 * lr_integrate with this model, rank and precision, bitwise the same result --
 * with no context, no caller workspace and no allocation of any kind.  Its
 * workspace is a fixed 16 MiB array in device memory inside the library (one
 * per GPU, held until the process ends); shapes whose persistent-path
 * workspace exceeds it return LR_ERR_OOM (N = 2000 at M = 20 takes 3.7 MiB,
 * N = 3000 at M = 32 11.6 MiB), shapes without a persistent configuration
 * LR_ERR_ARG.  Arguments and
 * records as lr_init and lr_integrate.  d_status (device, 2 int64, may be
 * NULL) receives {status code, failing step} at the end of the enqueued work:
 * the device-side errors lr_status would report.  Enqueued on `stream` (NULL:
 * the null stream).  Every call on a GPU uses that GPU's one array, which
 * keeps the last call's contents (every call re-initialises what it reads):
 * calls that overlap on one GPU -- on different streams or from different
 * threads -- race and must not be issued. */
int lr_integrate_noalloc(const lr_model_t* model, int32_t M, int32_t precision, const lr_pulse_t* pulse, double t0,
                         double dt, int64_t nsteps, lr_c64* d_B, int32_t obs_stride, double* d_obs,
                         int64_t* d_status, void* stream);

const char* lr_strerror(int code);
void lr_destroy(lr_ctx_t* ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent trajectories (e.g. pulse candidates x {g, e},
 * each with its own model dims, rank, drive, dt and step count) integrated
 * together.  Each trajectory is the lr_integrate problem above; results are
 * bitwise those of the same trajectory run alone in a batch of one (every
 * reduction has a fixed order that does not depend on the batch).
 * ------------------------------------------------------------------------ */
typedef struct {
  lr_model_t model;
  int32_t M;
  int32_t precision;        /* LR_FP64, LR_FP32 or LR_BF16X3 */
  lr_pulse_t pulse;
  double t0, dt;
  int64_t nsteps;
  lr_c64* d_B;              /* device, column-major N x M; in B(t_first), out B(t_first + nsteps dt) */
  int32_t obs_stride;       /* records as in lr_integrate (0: none) */
  int32_t step0;            /* index of the first step (>= 0): step n of this call runs from
                               t0 + (step0 + n) dt, so a trajectory continued over several
                               calls (t0 fixed, step0 advanced) sees bitwise the same stage
                               times, hence the same result, as in one call */
  double* d_obs;            /* device, (nsteps / obs_stride + 1) x LR_OBS_LEN(d_q) */
} lr_traj_t;

typedef struct lr_batch lr_batch_t;

/* Plan a batch (host only): validates every trajectory (as lr_init and
 * lr_integrate do), copies the descriptors and sizes the workspace.  The
 * device pointers inside the descriptors are used by lr_batch_run. */
int lr_batch_init(lr_batch_t** batch, const lr_traj_t* trajs, int32_t n);
/* lr_batch_init with schedule flags.  0 is lr_batch_init.  LR_BATCH_PACKED:
 * every trajectory (LR_FP64; LR_FP32 and LR_BF16X3 for model kinds 0 and 1,
 * see LR_BATCH_PACKED_MFMA64) with d_q d_f M <= LR_PACKED_MAX_LM (and whose
 * workgroup's LDS, about 16 (4 d_q d_f M + 2 M^2 + 2.5 d_q d_f) bytes, fits
 * 159 KiB) runs in a workgroup of its own (all of them in one launch per chunk of steps, as many
 * per CU as fit), which fills the GPU with many trajectories at once instead
 * of spreading each one over d_r workgroups; the other trajectories run as
 * without the flag.  A packed trajectory's result does not depend on the
 * batch either (fixed-order sums, one workgroup), but its rounding is not that
 * of the spread schedule: the two agree to the FP64 tolerances of lr_integrate.
 * Unknown flag bits: LR_ERR_ARG. */
#define LR_BATCH_PACKED 1
#define LR_PACKED_MAX_LM 1536
/* Packed schedule, Gram and cross products [G | C_1 | C_2] of model kinds 0
 * and 1: LR_FP32 and LR_BF16X3 trajectories form them on the matrix cores
 * (v_mfma 16 x 16 output tiles: LR_FP32 with the FP32 instruction and FP32
 * accumulation; LR_BF16X3 with three BF16 part products per real product and
 * FP32 accumulation for C_k, the FP64 instruction for G).  FP64 trajectories
 * form them on the vector ALU (one thread per entry block, rows in order), or
 * with LR_BATCH_PACKED_MFMA64 on the matrix cores with the FP64 instruction
 * (slower at M = 20: the tiles are padded to 32 x 64 and the FP64 matrix rate
 * equals the vector rate).  The stencil, the jump assembly, the solve and the
 * RK4 state are FP64 in every packed mode.  Model kind 2 and adaptive
 * batches: vector ALU, FP64 only. */
#define LR_BATCH_PACKED_MFMA64 2
/* Tile height of the spread schedule: resonator layers per workgroup
 * (1..255; 0 or absent: one).  A height whose tile does not fit the kernel's
 * register rows or LDS is lowered to the largest that fits.  Combined with the
 * other flags by |; the autotuner of the Python package searches it. */
#define LR_BATCH_SPREAD_LAYERS(k) ((int32_t)((k) & 0xff) << 8)
/* Layer-split packed trajectories, for latency when few trajectories are in
 * flight: with LR_BATCH_PACKED (or in an adaptive batch), every LR_FP64
 * packed trajectory runs on p workgroups (2..255, at most d_r; 0 or absent:
 * one), each over a contiguous range of about d_r / p resonator layers.  After
 * every pass the parts' Gram and cross terms are summed in a fixed order
 * (partials, group barrier, a slice reduction per part, group barrier), and
 * every part solves the same M x M system; model kind 2 pairs the layers across
 * a part boundary after the part above has published its first layer.  The
 * parts of a trajectory and of the batch's other split trajectories run
 * co-resident (cooperative launches, as in the spread schedule; not captured by
 * lr_batch_graph), and their bounded waits end in LR_ERR_TIMEOUT as there.
 * The result depends on p only through the rounding of the sums over the parts
 * (it agrees with the one-workgroup form to the FP64 tolerances of
 * lr_integrate).  Reduced-precision trajectories stay one workgroup each.  A
 * trajectory whose p parts cannot be co-resident: LR_ERR_ARG at lr_batch_bind. */
#define LR_BATCH_PACKED_PARTS(p) ((int32_t)((p) & 0xff) << 16)
int lr_batch_init_ex(lr_batch_t** batch, const lr_traj_t* trajs, int32_t n, int32_t flags);
/* Adaptive-step batch (main text, "Computational performance": the paper's
 * solver has an adaptive time step): every trajectory takes Dormand-Prince
 * 5(4) steps of its own size in the packed schedule, with the error norm
 * sqrt(mean_i |e_i|^2 / (atol + rtol max(|y_i|, |ynew_i|))^2) over the N M
 * entries of B and the step controller min(5, max(0.2, 0.9 err^(-1/5))).
 * For an adaptive trajectory, dt is the output grid and the first trial
 * step: it is integrated from t0 + step0 dt to t0 + (step0 + nsteps) dt and
 * recorded every obs_stride grid points (steps land on those times and on no
 * others, whatever the other trajectories of the batch; with obs_stride 0, on
 * the end time only).  Every
 * trajectory must qualify for LR_BATCH_PACKED (LR_FP64, layer size), and
 * rtol, atol > 0; else LR_ERR_ARG.  A step size below 1e-14 max(1, |t|), or
 * more than 2^22 attempts within one output interval, stops the trajectory
 * with LR_ERR_STEP. */
int lr_batch_init_adaptive(lr_batch_t** batch, const lr_traj_t* trajs, int32_t n, double rtol, double atol);
/* lr_batch_init_adaptive with schedule flags: 0, LR_BATCH_PACKED or
 * LR_BATCH_PACKED_PARTS(p) (layer-split trajectories); other bits: LR_ERR_ARG. */
int lr_batch_init_adaptive_ex(lr_batch_t** batch, const lr_traj_t* trajs, int32_t n, int32_t flags, double rtol,
                              double atol);
/* Accepted and rejected step counts of an adaptive batch after lr_batch_run
 * (arrays of n, caller order; synchronises).  LR_ERR_STATE for other batches. */
int lr_batch_adaptive_stats(lr_batch_t* batch, int64_t* accepted, int64_t* rejected);
size_t lr_batch_workspace_bytes(const lr_batch_t* batch);
int lr_batch_bind(lr_batch_t* batch, void* d_workspace, size_t bytes, void* stream);
/* Enqueue the integration of every trajectory of the batch on the bound
 * stream.  Trajectories are packed into co-resident groups and run
 * concurrently, group after group. */
int lr_batch_run(lr_batch_t* batch);
/* Graph mode for batches whose trajectories all run in the packed schedule
 * (LR_BATCH_PACKED or adaptive): while on, the first lr_batch_run captures its
 * whole launch sequence on the bound stream into a HIP graph and every call
 * replays it.  A replay integrates the same problems again from the current
 * contents of every d_B (descriptors, step counts and records as at
 * lr_batch_init); kernel timing (lr_batch_profile_*) is not recorded while on.
 * on = 0 drops the graph.  LR_ERR_STATE before lr_batch_bind, when the batch
 * is bound to the null stream (which cannot be captured), or when a
 * trajectory runs in the spread schedule or is layer-split
 * (LR_BATCH_PACKED_PARTS; their cooperative launches are not captured). */
int lr_batch_graph(lr_batch_t* batch, int32_t on);
/* Synchronise; per-trajectory status codes and failing step indices
 * (arrays of n, may be NULL).  Returns the first non-OK code or LR_OK. */
int lr_batch_status(lr_batch_t* batch, int32_t* codes, int64_t* failed_steps);
/* Kernel timing of a batch: while enabled, every chunk launch of the
 * persistent kernel made by lr_batch_run is bracketed by HIP events on the
 * bound stream (the first LR_PROFILE_MAX launches after enabling; enabling
 * again resets the count).  lr_batch_profile_read synchronises the stream and
 * returns the summed kernel time (ms) and the launch count. */
int lr_batch_profile_enable(lr_batch_t* batch, int32_t on);
/* lr_wait_limits for every spread-schedule and layer-split trajectory of a
 * bound batch (enqueued on the bound stream; applies to later lr_batch_run
 * calls; the one-workgroup packed and adaptive kernels have no group
 * barriers).  LR_ERR_STATE before lr_batch_bind. */
int lr_batch_wait_limits(lr_batch_t* batch, uint32_t spins, int32_t never);
int lr_batch_profile_read(lr_batch_t* batch, double* ms, int64_t* launches);
void lr_batch_destroy(lr_batch_t* batch);

#ifdef __cplusplus
}
#endif
#endif /* LR_H */
