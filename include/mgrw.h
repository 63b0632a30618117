/*
 * mgrw -- leading-order event reweighting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libmgrw.so.  The library evaluates, per event, the tree-level
 * squared matrix element |M|^2 (arXiv:2312.07440, Sec. 2.1, eq. (1): the
 * amplitude factor of the event weight) from helicity amplitudes, and the
 * reweighted weight
 *
 *     W' = W |M'|^2 / |M|^2                     (Sec. 2.2, eq. (3))
 *
 * for a batch of events and a set of model-parameter points, following the
 * reweighting procedure of Sec. 3.2 (1: input parameters, 3: original
 * amplitudes, 4: overwrite parameters, 5: new amplitudes, 6: new weight,
 * 7: repeat for all parameter sets, 8: return weights).  Event parsing
 * (step 2) is the caller's: events arrive as device arrays.
 *
 * Conventions shared by all calls:
 *  - Momenta are DEVICE pointers to float64 in "structure of arrays" layout:
 *    mom[(i*4 + mu)*n_events + e] is component mu = (E, px, py, pz), in GeV,
 *    of external particle i of event e, in the partonic centre-of-mass frame
 *    (incoming partons along +z and -z).  Particle order follows the process
 *    name: (e+, e-, mu+, mu-) or (g, g, t, tbar, g, ...).
 *  - Event-sized inputs and outputs are DEVICE pointers owned by the caller
 *    (for instance PyTorch tensors); the library never frees them.  Any
 *    n_events >= 0 is accepted (no padding); n_events == 0 launches nothing.
 *  - `stream` is a hipStream_t (NULL: the default stream).  Evaluation calls
 *    are asynchronous and stream-ordered; argument errors are reported before
 *    anything is launched, device faults surface at a later synchronisation.
 *    The double-precision pipeline of g g -> t tbar g g g also runs kernels on
 *    three library-owned streams of the device (default priority, created on
 *    first use, kept until the process ends), forked from and joined back
 *    into `stream` with events, so the call stays ordered on `stream`.
 *  - Return values are mgrw_status codes; on a non-OK status the calling
 *    thread's mgrw_last_error() describes it.  No exception crosses the ABI.
 *  - A process handle is not thread-safe; distinct handles are independent.
 */
#ifndef MGRW_H
#define MGRW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgrw_process mgrw_process;

enum {
    MGRW_OK = 0,
    MGRW_ERR_ARG = -1,          /* invalid argument (null, range, layout) */
    MGRW_ERR_UNSUPPORTED = -2,  /* process/precision combination not built */
    MGRW_ERR_DEVICE = -3,       /* HIP runtime error */
    MGRW_ERR_ALLOC = -4,        /* host allocation failed */
    MGRW_ERR_STATE = -5         /* call not valid in the handle's state */
};
typedef int mgrw_status;

/* Processes (tree level, Standard Model couplings; kappa scales every
 * top-top-gluon vertex).  Particle order in the momentum array: as written,
 * e.g. (e+, e-, mu+, mu-), (g, g, t, tbar, g, ...), (e+, e-, a, a, a, a, a). */
enum {
    MGRW_EE_MUMU = 1,    /* e+ e- -> mu+ mu- via photon and Z           */
    MGRW_GG_TT = 2,      /* g g -> t tbar                               */
    MGRW_GG_TTG = 3,     /* g g -> t tbar g                             */
    MGRW_GG_TTGG = 4,    /* g g -> t tbar g g                           */
    MGRW_GG_TTGGG = 5,   /* g g -> t tbar g g g                         */
    MGRW_EE_5A = 6       /* e+ e- -> 5 photons, massless electron (the
                            process of the paper's timing study, Table 1);
                            120 diagrams; parameter: alpha            */
};

/* Arithmetic of the amplitude chains. */
enum {
    MGRW_FP64 = 0,       /* everything in double                              */
    MGRW_MIXED = 1       /* wavefunctions, vertex chains and colour sum in float;
                            kinematics, propagator denominators, helicity sum and
                            the ratio of eq. (3) in double                        */
};

/* One model-parameter point (runtime-modifiable parameters, Sec. 3.2: the
 * procedure only holds for parameters that can be changed at run time).
 * e+e- uses alpha, sw2, mz, wz; QCD processes use alphas, mt, kappa_ttg.
 * wt (top width) must be 0: internal top lines are off shell in these
 * processes and gauge invariance at kappa = 1 requires it. */
typedef struct {
    double alpha;      /* QED coupling alpha                                  */
    double sw2;        /* sin^2(theta_W)                                      */
    double mz, wz;     /* Z mass and width, GeV                               */
    double alphas;     /* strong coupling alpha_s                             */
    double mt, wt;     /* top mass and width, GeV                             */
    double kappa_ttg;  /* scale factor of the top-top-gluon coupling          */
} mgrw_params;

#define MGRW_MAX_POINTS 64

/* Create a handle for `proc` at arithmetic `prec` with base (original)
 * parameters `base` (host pointer, copied).  Step 1 of the procedure for the
 * original model.  Errors: MGRW_ERR_ARG (null out/base, unknown proc or prec,
 * non-finite or unphysical parameters), MGRW_ERR_UNSUPPORTED (e+e- in mixed
 * precision), MGRW_ERR_ALLOC. */
mgrw_status mgrw_create_process(int proc, int prec, const mgrw_params *base, mgrw_process **out);

/* Set the new parameter points (steps 1 and 4 of the procedure): `points` is
 * a HOST array of n_points in [1, MGRW_MAX_POINTS], copied before return;
 * later calls use the new set, calls already launched keep theirs.  External
 * masses (mt) must equal the base value: events are on shell for them and
 * the new phase space must lie inside the old one (Sec. 2.2).
 * Errors: MGRW_ERR_ARG. */
mgrw_status mgrw_set_params(mgrw_process *p, const mgrw_params *points, int32_t n_points);

/* |M|^2 of every event at one parameter point (steps 3 or 5): point = -1 is
 * the base point, 0 <= point < n_points a point of mgrw_set_params.
 * me_out: device float64[n_events].  Normalisation: averaged over incoming
 * spins and colours, summed over outgoing ones, divided by n! for n identical
 * outgoing gluons.  Errors: MGRW_ERR_ARG (null or host pointers, n_events < 0,
 * point out of range), MGRW_ERR_STATE (point >= 0 with no points set),
 * MGRW_ERR_DEVICE (launch failure). */
mgrw_status mgrw_eval_me(mgrw_process *p, const double *mom, int64_t n_events, int32_t point,
                         double *me_out, void *stream);

/* Reweight (steps 3-8): for every event e and new point k,
 *   w_out[k*n_events + e] = W_e * (|M_k|^2 / |M_base|^2),
 * W_e = w_in[e] (device float64[n_events]) or 1 when w_in is NULL; quiet NaN
 * where |M_base|^2 = 0 (eq. (3) requires |M|^2 != 0).  me_base_out (device
 * float64[n_events], may be NULL) receives |M_base|^2.  All points are
 * evaluated in full inside one kernel, so momenta are read once.
 * Errors: as mgrw_eval_me; MGRW_ERR_STATE when no points are set. */
mgrw_status mgrw_reweight(mgrw_process *p, const double *mom, const double *w_in, int64_t n_events,
                          double *w_out, double *me_base_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as mgrw_reweight, bit for bit, without any allocation.  The
 * per-event kinematics records and the list of events for the FP64
 * re-evaluation come from a 256 MiB device array inside the library (one per
 * GPU, held until the process ends); the events run in chunks whose buffers
 * fit it (about 2.5e5 events per chunk for g g -> t tbar g g).  The call
 * allocates nothing and records no kernel timing (mgrw_kernel_time_ms then
 * reports MGRW_ERR_STATE).  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads, other handles)
 * race and must be serialised by the caller; nothing from a previous call is
 * read.  The stream must belong to the current device.
 * Errors: as mgrw_reweight; MGRW_ERR_UNSUPPORTED for g g -> t tbar g g g (its
 * colour-flow buffers, about 2 MB per event, exceed the array) and device
 * ordinals above 63; MGRW_ERR_ARG for a stream of another device;
 * MGRW_ERR_DEVICE if the array's address cannot be obtained. */
mgrw_status mgrw_reweight_noalloc(mgrw_process *p, const double *mom, const double *w_in, int64_t n_events,
                                  double *w_out, double *me_base_out, void *stream);

/* mgrw_reweight for events and weights in HOST memory (procedure steps 2-8
 * with the transfers, which dominate small samples: Sec. 3.3).  mom
 * ([n_ext][4][n_events]), w_in ([n_events], may be NULL), w_out
 * ([n_points][n_events]) and me_base_out ([n_events], may be NULL) are host
 * arrays in the layouts of mgrw_reweight, owned by the caller.  The batch is
 * processed in chunks of `chunk` events (0: 2^18) on two streams of the
 * library's own, so one chunk's copies overlap the other's kernels; pinned
 * host memory makes the copies asynchronous (pageable memory works, without
 * the overlap).  Synchronous: returns when w_out is written.  The results
 * equal mgrw_reweight's bit for bit.  Errors: MGRW_ERR_ARG (null pointers,
 * n_events < 0, chunk < 0), MGRW_ERR_STATE (no points), MGRW_ERR_ALLOC,
 * MGRW_ERR_DEVICE. */
mgrw_status mgrw_reweight_host(mgrw_process *p, const double *mom, const double *w_in, int64_t n_events,
                               double *w_out, double *me_base_out, int64_t chunk);

/* Exact reweighting by the kappa polynomial.  Same contract and results (to
 * rounding) as mgrw_reweight, by a different evaluation: every diagram carries
 * g_s^n kappa^k with k its number of top-gluon vertices, so one evaluation per
 * helicity at unit couplings gives the amplitudes J_k of each power and
 *   |M|^2(g_s, kappa) = g_s^(2n) sum_{k,k'} kappa^(k+k') Re(J_k^+ CF J_k')
 * for every point at the cost of a few colour products: the work no longer
 * grows with the number of points.  Points may differ from the base in
 * alphas and kappa_ttg.  g g -> t tbar + 0..2 g.  Errors: as mgrw_reweight;
 * MGRW_ERR_UNSUPPORTED for other processes. */
mgrw_status mgrw_reweight_kpoly(mgrw_process *p, const double *mom, const double *w_in, int64_t n_events,
                                double *w_out, double *me_base_out, void *stream);

/* Static properties of the process: external particles, colour flows,
 * helicity configurations evaluated per event and point, Feynman diagrams.
 * Any output pointer may be NULL.  Errors: MGRW_ERR_ARG (null handle). */
mgrw_status mgrw_process_info(const mgrw_process *p, int *n_ext, int *n_flows, int *n_hel,
                              int *n_diagrams);

/* Options.  MGRW_OPT_LANE_MAPPING selects how events map onto the GPU's
 * lanes for the exact QCD kernels: MGRW_MAP_AUTO (default),
 * MGRW_MAP_EVENT_PER_LANE (one event per lane, helicities in a loop), or
 * MGRW_MAP_EVENT_PER_WAVE (one event per 64-lane wave, helicity
 * configurations on the lanes; processes with a multiple of 64 helicity
 * configurations only).  Results agree to rounding.
 *
 * MGRW_OPT_RESCUE_PPM (mixed precision, g g -> t tbar + 0..3 g): events in
 * which a gluon pair other than the two beams has |2 p_i.p_j| / s below
 * value * 1e-6 are evaluated a second time in FP64 and their results
 * replaced.  There the diagrams cancel strongly and single-precision
 * amplitudes lose up to about three more digits.  Default for mixed-precision
 * handles: 3000 (3e-3) for g g -> t tbar + 1..2 g, 1000 (1e-3) for
 * g g -> t tbar g g g (about 2 % of its events; its FP64 pipeline costs four
 * times the single-precision one), chosen from full-sample comparisons with
 * the FP64 kernels; 0 (off) otherwise; 0..1000000.
 * Applies to mgrw_eval_me, mgrw_reweight and mgrw_reweight_kpoly.
 *
 * MGRW_OPT_COLOUR_MFMA (0 or 1; g g -> t tbar g g g): 1 forms the colour sum
 * J^+ CF J on the matrix cores (bfloat16-split operands, float32
 * accumulation; results agree with the default VALU form to float32
 * rounding) after the last program part; default 0.
 *
 * MGRW_OPT_SURROGATE_INPUTS (53 or 25): input features of the surrogate that
 * mgrw_surrogate_train fits and mgrw_reweight_surrogate evaluates (events
 * in, not mgrw_surrogate_train_samples): 53 (default) = the 24 momentum
 * components over sqrt(s)/2, (kappa - 1)/0.2, and 2 p_i.p_j/s with its
 * logarithm for the 14 pairs other than the beams; 25 = the momentum
 * components and kappa only (the other columns zero).  A network must be
 * evaluated with the setting it was trained with.
 *
 * MGRW_OPT_KERNEL_TIMING (0 or 1): when 1, every launch records a pair of HIP
 * events on its stream around its amplitude kernel(s) (after the setup of
 * the kinematics, before the FP64 re-evaluation), read by
 * mgrw_kernel_time_ms.
 *
 * Errors: MGRW_ERR_ARG (unknown option or value), MGRW_ERR_UNSUPPORTED
 * (mapping or rescue not available for the process or precision),
 * MGRW_ERR_DEVICE (event creation failed). */
enum { MGRW_OPT_LANE_MAPPING = 1, MGRW_OPT_RESCUE_PPM = 2, MGRW_OPT_KERNEL_TIMING = 3, MGRW_OPT_COLOUR_MFMA = 4,
       MGRW_OPT_SURROGATE_INPUTS = 5 };
enum { MGRW_MAP_AUTO = 0, MGRW_MAP_EVENT_PER_LANE = 1, MGRW_MAP_EVENT_PER_WAVE = 2 };
mgrw_status mgrw_set_option(mgrw_process *p, int option, int64_t value);

/* Current value of an option (as mgrw_set_option takes it) in *value.
 * Errors: MGRW_ERR_ARG (null handle or value, unknown option). */
mgrw_status mgrw_get_option(const mgrw_process *p, int option, int64_t *value);

/* Device time in ms of the amplitude kernel(s) of the handle's most recent
 * launch (kernel timing on); waits for that launch to finish.  Errors:
 * MGRW_ERR_STATE (timing off or nothing launched since it was switched on),
 * MGRW_ERR_DEVICE. */
mgrw_status mgrw_kernel_time_ms(mgrw_process *p, double *ms);

/* Release the handle (NULL is ignored).  Work already launched with it is
 * unaffected: its parameters travelled with the launch.  The streams and
 * staging buffers of mgrw_reweight_host are released after their work ends. */
void mgrw_destroy_process(mgrw_process *p);

/* One reweight over a sample that mixes processes, such as the Born and
 * real-emission configurations of an NLO sample (g g -> t tbar and
 * g g -> t tbar g; the same tree-level machinery evaluates both, Sec. 4).
 * procs[0..n_procs-1] (1..8 handles, all with the same number of points P);
 * proc_index[e] (device, int32) selects event e's process; mom (device) holds
 * n_ext_max momentum rows per event, mom[(i*4+mu)*N + e], of which a process
 * with n_ext particles reads rows 0..n_ext-1 in its own particle order.
 * w_out [P][N] and me_base_out (nullable) as in mgrw_reweight; each event's
 * results are those mgrw_reweight gives for it with its process's handle.
 * The events of each process are gathered into a contiguous batch on the
 * device and reweighted there; the call synchronises the stream once, to
 * read the per-process counts.  Errors: MGRW_ERR_ARG (sizes, differing P,
 * indices outside [0, n_procs)), MGRW_ERR_STATE, MGRW_ERR_DEVICE, and those of
 * mgrw_reweight. */
mgrw_status mgrw_multi_reweight(mgrw_process *const *procs, int n_procs, const double *mom, int n_ext_max,
                                const int32_t *proc_index, const double *w_in, int64_t n_events, double *w_out,
                                double *me_base_out, void *stream);

/* ------------------------------------------------------------------------
 * Les Houches event files: steps 2 (events in) and 8 (weights out) of the
 * reweighting procedure (Sec. 3.2).  Host memory, host code.
 *
 * mgrw_lhe_open reads a whole file; its text is kept so that mgrw_lhe_write
 * reproduces every byte of it and only adds the new weights.
 * mgrw_lhe_events fills mom[(i*4+mu)*N + e] (the layout of mgrw_reweight,
 * host memory, N = mgrw_lhe_info's count) in the particle order of process
 * proc: the event's incoming (status -1) and outgoing (status +1) particles
 * are matched to the process's slots by PDG code in order of appearance
 * (intermediate particles are skipped), and every event is boosted along the
 * beam axis to the frame in which its incoming momenta sum to zero (the frame
 * of the amplitudes' polarisation vectors).  w (nullable) receives each
 * event's XWGTUP.  Errors: MGRW_ERR_ARG with the file, line or event and the
 * reason (unreadable file, malformed event, particle content that does not
 * match the process, incoming partons off the beam axis).
 * mgrw_lhe_write writes the file with, in every event, one
 * <wgt id='ids[k]'> w_new[k*N + e] </wgt> per point (17 significant digits)
 * added to the event's <rwgt> block (created if absent) and the ids declared
 * in the header's <initrwgt> block (created inside <header> if absent); it
 * writes path.part and renames it, so a failed write leaves no partial file.
 * Ids must be non-empty and free of quotes, markup and newlines. */
typedef struct mgrw_lhe mgrw_lhe;
mgrw_status mgrw_lhe_open(const char *path, mgrw_lhe **out);
mgrw_status mgrw_lhe_info(const mgrw_lhe *h, int64_t *n_events);
mgrw_status mgrw_lhe_events(const mgrw_lhe *h, int proc, double *mom, double *w);
mgrw_status mgrw_lhe_write(const mgrw_lhe *h, const char *path, const double *w_new, int n_points,
                           const char *const *ids);
void mgrw_lhe_close(mgrw_lhe *h);

/* ------------------------------------------------------------------------
 * Learned surrogate of the reweight factor.
 *
 * A multilayer perceptron predicts y = log(|M_k|^2 / |M_base|^2) for an event
 * and a parameter point k: inputs are the 24 momentum components of the
 * event divided by sqrt(s)/2, kt = (kappa_k - 1)/0.2, and for the 14 particle
 * pairs other than the two beams v = 2 p_i.p_j / s and log v
 * (MGRW_SURROGATE_N_FEATURES = 53 values); four hidden layers of
 * 256 SiLU units (bfloat16 weights, float32 accumulation on the matrix
 * cores); the output is yhat = (kappa_k - 1) * h, h the last linear unit, so
 * the prediction is exact at kappa = 1.  Surrogate weights W~' = W exp(yhat).
 * A random audit subset of events is evaluated exactly (eq. (3)) and serves
 * as a control variate for the sums of weights.  QCD processes only; the
 * base point must have kappa_ttg = 1 (where the prediction is exact) and the
 * points must differ from it only in kappa_ttg (MGRW_ERR_UNSUPPORTED
 * otherwise).
 *
 * Parameters (float32, MGRW_SURROGATE_N_PARAMS values) in this order:
 * W1[256][64] (input columns 53..63 unused, zero), b1[256], W2[256][256],
 * b2[256], W3[256][256], b3[256], W4[256][256], b4[256], w5[256], b5[1];
 * W[out][in].
 * ------------------------------------------------------------------------ */

#define MGRW_SURROGATE_N_PARAMS 214273
#define MGRW_SURROGATE_N_FEATURES 53

typedef struct {
    int32_t epochs;      /* passes over the training samples                     */
    int32_t batch;       /* samples (event, point) per Adam step, multiple of 64 */
    double lr;           /* Adam step size                                       */
    double lr_decay;     /* step-size factor applied after each epoch            */
    uint64_t seed;       /* initialisation and shuffling                         */
} mgrw_train_config;

/* Train the surrogate on n_events events (device momenta as for
 * mgrw_reweight) at the handle's current points: the exact kernels label every
 * (event, point) pair (the kappa-polynomial evaluation of
 * mgrw_reweight_kpoly where the process has it, exact up to rounding), then
 * the network is fitted by mean-squared error with Adam on shuffled batches
 * (a keyed permutation of the samples per epoch), all on the device.  A previous network is replaced, starting from a
 * seeded initialisation.  loss_out (host, may be NULL) receives the mean
 * training loss of each epoch.  Synchronous.  Errors: MGRW_ERR_ARG,
 * MGRW_ERR_UNSUPPORTED (e+e- process, or points that change more than
 * kappa_ttg), MGRW_ERR_STATE (no points), MGRW_ERR_DEVICE, MGRW_ERR_ALLOC. */
mgrw_status mgrw_surrogate_train(mgrw_process *p, const double *mom, int64_t n_events,
                                 const mgrw_train_config *cfg, double *loss_out, void *stream);

/* Train the surrogate on m given samples instead of exact labels (device
 * arrays, the layout of mgrw_surrogate_fwd_bwd): features x[m][53] (float32,
 * rounded to bfloat16 like the computed ones), kd[m] (the factor the output
 * unit is multiplied by), targets y[m].  Same network, initialisation, batches
 * and Adam as mgrw_surrogate_train; the handle's process and points are not
 * used (any handle may hold the network).  For fitting targets computed
 * elsewhere and for checking the training on a known function.  Synchronous.
 * Errors: MGRW_ERR_ARG (null pointers, m outside [batch, 2^31), bad
 * configuration), MGRW_ERR_DEVICE, MGRW_ERR_ALLOC. */
mgrw_status mgrw_surrogate_train_samples(mgrw_process *p, const float *x, const float *kd, const float *y, int64_t m,
                                         const mgrw_train_config *cfg, double *loss_out, void *stream);

/* Reweight with the surrogate and an exact audit.  Every event gets
 * w_out[k*n_events + e] = W_e exp(yhat); events selected by the audit (a
 * counter-based hash of (seed, e) below audit_fraction, in (0, 1]) are
 * evaluated exactly and receive the exact W'.  audit_stats (host,
 * [n_points][5], may be NULL) receives per point: the control-variate estimate
 * of sum_e W'_e (surrogate sum + (exact - surrogate) summed over the audit /
 * audit_fraction), the surrogate sum, the audited mean |W~'/W' - 1|, its
 * standard error, and the number of audited events.  The mean and its error
 * are taken over the audited events with a finite, non-zero exact weight
 * (a zero input weight makes both weights zero; |M|^2 = 0 at the base makes
 * the exact one NaN, eq. (3)); with none of those the mean is 0.  If the
 * audited mean error of any point exceeds max_audit_error (or is NaN) the
 * whole batch is recomputed exactly and *fell_back (may be NULL) is set to 1.
 * Scratch memory is allocated and freed in the stream's order; the call
 * synchronises the stream once, to read the audit statistics.
 * Errors: as mgrw_reweight (host pointers among mom, w_in, w_out:
 * MGRW_ERR_ARG); MGRW_ERR_STATE if no surrogate is trained. */
mgrw_status mgrw_reweight_surrogate(mgrw_process *p, const double *mom, const double *w_in, int64_t n_events,
                                    double audit_fraction, uint64_t seed, double max_audit_error,
                                    double *w_out, double *audit_stats, int *fell_back, void *stream);

/* Copy the surrogate parameters to / from a host float array of
 * MGRW_SURROGATE_N_PARAMS values (checkpointing, tests).  _get needs a
 * trained or loaded surrogate (MGRW_ERR_STATE otherwise); _set creates one. */
mgrw_status mgrw_surrogate_get(const mgrw_process *p, float *params);
mgrw_status mgrw_surrogate_set(mgrw_process *p, const float *params);

/* Checkpoint the surrogate to a file and back.  Format: the 8 bytes
 * "MGRWSUR1", uint32 n_params (= MGRW_SURROGATE_N_PARAMS), uint32 0, then the
 * n_params float32 parameters in the order above, all little-endian.  _save
 * needs a trained or loaded surrogate (MGRW_ERR_STATE), writes path.part and
 * renames it.  _load reads and checks the whole file (MGRW_ERR_ARG: missing,
 * short, wrong magic or count) before it replaces the handle's network, as
 * _set does; Adam moments start from zero.  Synchronous. */
mgrw_status mgrw_surrogate_save(const mgrw_process *p, const char *path);
mgrw_status mgrw_surrogate_load(mgrw_process *p, const char *path);

/* One forward and backward pass over m given samples (device arrays):
 * x[m][MGRW_SURROGATE_N_FEATURES] features, kd[m] = kappa - 1, y[m] targets; pred[m] (device)
 * receives yhat, grad (host, MGRW_SURROGATE_N_PARAMS floats) the gradient of
 * the mean squared error, loss (host) its value.  m is a multiple of 64.
 * The same kernels as training.  Errors: MGRW_ERR_ARG, MGRW_ERR_STATE. */
mgrw_status mgrw_surrogate_fwd_bwd(mgrw_process *p, const float *x, const float *kd, const float *y, int64_t m,
                                   float *pred, float *grad, double *loss, void *stream);

/* Text describing the calling thread's last non-OK status ("" if none). */
const char *mgrw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGRW_H */
