/*
 * qedspin.h -- C ABI of the MI355X (gfx950) implementation of the spin- and
 * polarization-resolved strong-field QED particle step of Qian, Seipt, Vranic,
 * Grismayer, Ridgers and Thomas, "A Fully Spin and Polarization Resolved Strong Field
 * QED Algorithm for Particle-in-Cell Codes" (arXiv 2511.08929).
 *
 * The step, per electron or positron (NLC section and its flow chart): Lorentz push and
 * T-BMT spin rotation; chi_e and the rest-frame basis (eps, beta, k) (basis section);
 * the spin-weighted emission rate from the spin-up / spin-down rate tables; a
 * Philox4x32-10 draw against W dt; on emission the photon energy from the spin-up or
 * spin-down inverse CDF, recoil, collapse of the lepton spin onto its quantization axis
 * and of the photon Stokes vector onto its polarization axis, stored as a P-vector
 * (photon-polarization section); without emission the no-transition spin update
 * (non-transition section).  Per photon (NBW section): ballistic move, chi_gamma, the
 * Stokes vector decoded from the P-vector in the local basis, the xi3-weighted pair rate,
 * the pair's momentum split, correlated electron / positron spins, or the no-pair
 * polarization update.
 *
 * Units: time in 1/omega_r, length in c/omega_r, momenta in m c, fields in
 * m c omega_r / e; eps_r = hbar omega_r / (m c^2).  Spin and P-vectors are lab-frame
 * 3-vectors.
 *
 * Conventions that hold for every entry point:
 *  - All particle pointers are DEVICE pointers owned by the caller; arrays are SoA, one
 *    array per component, element type double (QED_F64 tables) or float (QED_F32 tables).
 *  - Counts live on the device (int64).  Kernels process [0, *d_count) and append at
 *    *d_count; appends never write at or beyond `capacity`: the excess is dropped and
 *    counted in qed_counters.n_capacity_overflow.
 *  - Calls only enqueue work on the given stream and return; the status reports host-side
 *    argument checks and launch errors.  Device-side conditions go to qed_counters
 *    (device memory, caller-owned, accumulated, never reset by the library).
 *  - No call allocates device memory except qed_init_tables; scratch memory is the
 *    caller-provided workspace of at least qed_workspace_size() bytes.
 *  - Appends are order-preserving: new photons in increasing emitter index, new pairs in
 *    increasing photon index, so results are bitwise reproducible run to run.
 *  - Random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *    (id low, id high, step, channel).  Lepton id = (species << 62) | index; photon id =
 *    2^63 | (parent species << 61) | (round << 57) | ((parent index mod 2^33) << 24) |
 *    (step mod 2^24), round = the sub-cycling round (QED_SUBCYCLE; 0 otherwise).
 */
#ifndef QEDSPIN_H
#define QEDSPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *qed_stream;   /* a hipStream_t (NULL = default stream) */

typedef enum {
    QED_OK = 0,
    QED_ERR_INVALID = -1,     /* bad argument (NULL pointer, size, precision mismatch ...) */
    QED_ERR_HIP = -2,         /* a HIP runtime call or kernel launch failed */
    QED_ERR_CAPACITY = -3,    /* workspace too small */
    QED_ERR_UNSUPPORTED = -4  /* unknown field model or flag combination */
} qed_status;

typedef enum { QED_F64 = 0, QED_F32 = 1 } qed_precision;

/* Physics switches (the paper's per-effect toggles used in its verification runs). */
enum {
    QED_PUSH = 1u << 0,        /* Lorentz (Boris) push inside qed_emit before the QED step */
    QED_TBMT = 1u << 1,        /* T-BMT spin rotation in the push */
    QED_EMIT = 1u << 2,        /* nonlinear Compton emission */
    QED_RECOIL = 1u << 3,      /* p <- (1 - lambda) p on emission */
    QED_SPIN = 1u << 4,        /* lepton spin collapse on emission */
    QED_NOEMIT = 1u << 5,      /* no-transition spin update of non-emitters */
    QED_PHOTON_POL = 1u << 6,  /* photon Stokes collapse (else unpolarized photons) */
    QED_MEAN = 1u << 7,        /* mean-value mode: s_f = g/w, xi = F(s_f=0)/w, pair spins j/w0 */
    QED_PAIR = 1u << 8,        /* nonlinear Breit-Wheeler pair creation */
    QED_NOPAIR = 1u << 9,      /* no-transition polarization update of surviving photons */
    QED_PAIR_SPIN = 1u << 10,  /* correlated pair spins (else unpolarized pairs) */
    QED_OPTICAL_DEPTH = 1u << 11, /* emission decided by the optical depth (decision-making overview):
                                  tau += W dt in FP64, emission when tau >= tau* = -ln(1 - u), u from
                                  Philox channel 4; the leptons' tau / tau_target arrays are required */
    QED_REJECTION = 1u << 12,  /* emission decided and lambda sampled together by rejection
                                  (spectrum-sampling section): the candidate lambda = r1^3 is accepted
                                  when r2 < 3 r1^2 dW/dlambda dt, dW/dlambda the spectrum of the
                                  lepton's spin state; no inverse-CDF table is read for the emission.
                                  Not with QED_OPTICAL_DEPTH (QED_ERR_INVALID) */
    QED_G_CHI = 1u << 13,      /* T-BMT with the field-dependent anomalous moment (loop appendix: the
                                  Scorer-function term of the one-loop self-energy): a_e is scaled by
                                  a(chi)/a(0) = 2 pi int_0^inf du/(1+u)^3 z Gi(z), z = (u/chi)^(2/3),
                                  at the Boris mid-step chi (momentum (u- + u+)/2, energy gamma-),
                                  from a table built by qed_init_tables: ln a(chi)/a(0) at 64 nodes per
                                  decade of chi from 1e-7 to 1e4, 4-point Lagrange in ln chi; 1 below
                                  chi = 1e-7, the chi^(-2/3) law above 1e4.  a_e = alpha/(2 pi) gives
                                  the one-loop moment, a_e = 0 keeps g = 2 */
    QED_SUBCYCLE = 1u << 14    /* per-particle sub-cycling of the lepton QED part where the per-step
                                  draw needs W dt << 1 (decision-making section): after the push a
                                  lepton takes m sub-steps of dt/m, m the smallest power of two with
                                  W_s dt / m <= 0.1 (at most 16), W_s dt at the state after the push;
                                  the sub-steps run in 16 rounds (a lepton takes one in every
                                  16/m-th), each the whole QED part at its current chi and spin, with
                                  Philox channels offset by 16 x round and the round in the photon id;
                                  a round's photons follow the previous round's.  qed_emit runs the
                                  rounds as 16 launches of its three kernels; a plan runs them in one
                                  launch of its own (each sub-cycled lepton takes all its sub-steps
                                  there, and its photons, kept per slot and counted per round, are
                                  stored in that order by the processing pass), with the same
                                  results bit for bit.  Not with QED_OPTICAL_DEPTH or QED_REJECTION
                                  (QED_ERR_INVALID), nor in a plan with a learned inverse CDF
                                  (QED_ERR_UNSUPPORTED).  Leptons below W dt = 0.1 step exactly as
                                  without it */
};

/* Field models evaluated at each particle. */
enum {
    QED_FIELD_UNIFORM = 0,     /* E = E0, B = B0 */
    QED_FIELD_PLANE_LP = 1,    /* E0, B0 plus a linearly polarized wave along -x:
                                  E_y = a0 g(phi) cos(phi), B_z = -E_y, phi = t + x,
                                  g = sin^2(pi phi / phase_len) on [0, phase_len] (1 if phase_len = 0) */
    QED_FIELD_GRID2D = 2,      /* E0, B0 plus a static field on a periodic 2-D grid in (x, y): six FP32
                                  device arrays Ex, Ey, Ez, Bx, By, Bz of nx * ny nodes, node (i, j) at
                                  (x0 + i dx, y0 + j dy), index j * nx + i; bilinear interpolation
                                  (particles need x[0] and x[1]).  The arrays are read at every step;
                                  a plan copies them into its own node-interleaved layout at the
                                  start of each of its steps (the plan allocates 32 bytes per node) */
    QED_FIELD_ROTATING_E = 3   /* E0, B0 plus a uniform electric field of magnitude a0 rotating in the
                                  (x, y) plane at the reference frequency: E_x = a0 cos t,
                                  E_y = a0 sin t (the 0-D cascade setup of the polarized-cascade
                                  section); no position needed */
};

/* Rate / inverse-CDF table grid: nodes uniform in ln chi and in rho = ln(r/(1-r)).
   Index 0 = nonlinear Compton (chi_e), 1 = Breit-Wheeler (chi_gamma). */
typedef struct {
    int    n_chi[2];
    double lnchi0[2];
    double dlnchi[2];
    int    n_rho;
    double rho0, drho;
} qed_table_grid;

typedef struct {
    qed_table_grid grid;
    qed_precision  precision;   /* element type of every particle array used with these tables */
} qed_table_params;

typedef struct qed_tables_s *qed_tables;   /* opaque, library-owned device tables */

typedef struct {
    int64_t  capacity;          /* elements allocated in every array */
    int64_t *d_count;           /* device: live leptons; appends go here */
    int      species;           /* 0 = electron (charge -1), 1 = positron (+1) */
    void    *x[3];              /* position components; x[i] may be NULL if the field model
                                   does not depend on coordinate i (then it is not advanced) */
    void    *p[3];              /* momentum / (m c) */
    void    *s[3];              /* spin vector, |s| <= 1 */
    double  *tau, *tau_target;  /* optical depth and its target, FP64 in both precisions (NULL unless
                                   QED_OPTICAL_DEPTH); a target <= 0 is drawn at the particle's next step;
                                   pair-born leptons start at 0, 0 */
} qed_leptons;

typedef struct {
    int64_t   capacity;
    int64_t  *d_count;          /* device: photons stored (dead slots included) */
    int64_t  *d_count_prev;     /* device: photons that qed_pair steps; qed_pair sets it to
                                   *d_count when it finishes, so photons born later in the same
                                   step wait for the next one */
    void     *x[3];             /* may be NULL as for leptons */
    void     *k[3];             /* momentum hbar k / (m c) */
    void     *P[3];             /* P-vector (photon-polarization section) */
    uint64_t *id;               /* 0 marks a dead slot (decayed, retired or never stored) */
} qed_photons;

typedef struct {
    int    kind;
    double E0[3], B0[3];
    double a0, phase_len;
    const float *grid[6];       /* QED_FIELD_GRID2D only (device pointers, caller-owned) */
    int    nx, ny;
    double dx, dy, x0, y0;
} qed_fields;

typedef struct {
    double   t;                 /* time at the start of the step */
    double   dt;
    double   a_e;               /* anomalous magnetic moment in T-BMT */
    double   eps_r;
    double   chi_e_min, chi_e_max;  /* no QED below min; lookups clamped above max */
    double   chi_g_min, chi_g_max;
    double   k_retire;          /* photons with |k| below this are stored as dead slots / retired */
    int64_t  step;              /* Philox counter word */
    uint64_t seed;              /* Philox key */
    uint32_t flags;
    const int64_t *d_clock;     /* optional device step offset c (NULL = 0): the launch uses step + c and
                                   t + c dt, so one recorded sequence of calls (a HIP graph) can be
                                   replayed every step; advance it with qed_clock_advance */
} qed_step_params;

typedef struct {                /* device-resident, accumulated */
    unsigned long long n_emit, n_pair, n_prob_clamped, n_chi_clamped, n_norm_clamped,
                       n_capacity_overflow, n_retired,
                       n_lepton_steps,   /* leptons stepped by qed_emit */
                       n_photon_steps,   /* live photons stepped by qed_pair */
                       n_photon_qed,     /* of those, photons with chi_gamma >= chi_g_min (full NBW step) */
                       n_nonfinite;      /* particle-steps with a NaN or infinity in their inputs: a
                                            lepton whose x, p or s is not finite keeps its stored state
                                            (no push, no QED); one whose grid field at t is not finite is
                                            not pushed, one whose grid field at t + dt is not finite is
                                            pushed without the QED part; a photon whose k or x is not
                                            finite (or whose k is 0) becomes a dead slot; one whose P
                                            is not finite takes its QED part as unpolarized (P = 0); one
                                            in a non-finite grid field gets no QED part.  The step
                                            writes no NaN or infinity of its own.  Analytic field models
                                            take finite parameters of magnitude below 1e30 only
                                            (QED_ERR_INVALID otherwise).  A state is tested through the
                                            sum of its components, so magnitudes beyond a ninth of the
                                            element type's range also count as non-finite */
} qed_counters;

typedef struct {
    const char *name;           /* kernel name (library-owned string) */
    long long   calls;
    double      total_ms;       /* sum of kernel durations: start and stop events stamped by each dispatch */
} qed_kernel_time;

/* Build the rate tables ln int_0^1 w dlam (spin-down, spin-up; xi3 = -1, +1; the pair rows hold
   ln int w dlam + 8/(3 chi_gamma), which takes out the exponential fall of the pair rate at small
   chi_gamma and leaves a row that 4-point interpolation follows to 1e-8) and inverse-CDF
   tables nu = ln(lam/(1-lam)) at rho = ln(r/(1-r)) on the given grid, by quadrature on the GPU
   (NLC section: rate and ICDF tabulated only for s_beta = -1, +1; NBW section: only for
   xi3 = -1, +1).  Allocates device memory; synchronizes the stream.  Returns QED_ERR_INVALID
   for a NULL pointer or a grid with fewer than 4 nodes per axis. */
qed_status qed_init_tables(const qed_table_params *params, qed_stream stream, qed_tables *out);

/* Text of the HIP error behind the most recent QED_ERR_HIP returned on this thread
   ("" if none).  The string is owned by the library. */
const char *qed_last_error(void);

/* Copy the g-factor table of QED_G_CHI to host memory: ln(a(chi)/a(0)) at ln chi = ln 1e-7 +
   i ln(10)/64, i < *n (705).  Either pointer may be NULL (then that part is skipped); host
   pointers, synchronous. */
qed_status qed_tables_download_gfac(qed_tables tables, double *lngfac, int64_t *n);

/* Release the tables (device memory).  Safe on NULL. */
qed_status qed_free_tables(qed_tables tables);

/* Copy the FP64 tables to host memory (layout [4 channels][n_chi][...], channels NLC-down,
   NLC-up, NBW-minus, NBW-plus; the pair rate rows with their + 8/(3 chi) as stored).  Sizes in elements are returned when the pointers are NULL. */
qed_status qed_tables_download(qed_tables tables, double *lnrate, int64_t *n_lnrate,
                               double *nu, int64_t *n_nu);

/* Bytes of workspace qed_emit / qed_pair / qed_compact need for sets of up to
   max_particles elements (leptons or photons, whichever is larger). */
size_t qed_workspace_size(int64_t max_particles);

/* Lorentz (Boris) push with fields at (x, t), T-BMT rotation (if QED_TBMT; with QED_G_CHI the
   anomalous moment from the tables' g-factor table), then x += v dt, for leptons [0, *d_count).
   In place.  A lepton whose state or fields are not finite is left as stored (not counted: this
   call takes no counters). */
qed_status qed_push_spin(const qed_leptons *leptons, const qed_fields *fields,
                         const qed_step_params *params, qed_tables tables, qed_stream stream);

/* NLC step for leptons [0, *d_count): with QED_PUSH, first the push of qed_push_spin with
   fields at t; then QED with fields at t + dt.  Emitted photons are appended to `photons`
   (dead slots, id = 0, for photons below k_retire).  In place on the leptons. */
qed_status qed_emit(qed_tables tables, const qed_leptons *leptons, const qed_fields *fields,
                    const qed_step_params *params, const qed_photons *photons,
                    qed_counters *d_counters, void *workspace, size_t workspace_bytes,
                    qed_stream stream);

/* qed_emit without any allocation, for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
   results as qed_emit, with the workspace taken from a static device array of
   QED_NOALLOC_SCRATCH_BYTES held by the library on each GPU it runs on until the process ends.
   Sets of capacity up to QED_NOALLOC_MAX_LEPTONS only; a larger capacity returns QED_ERR_CAPACITY
   (text in qed_last_error) before anything is enqueued.  No hipMalloc, hipFree or allocating
   library call is made; the array's device address is looked up once per device at the first
   call on it (with that device current).  All calls on one GPU share that GPU's array: calls
   that overlap on one GPU (other streams, other threads) race and must be ordered by the caller.
   Nothing in the array needs clearing between calls (every word a step reads is written earlier
   in the same step). */
#define QED_NOALLOC_MAX_LEPTONS 4194304
#define QED_NOALLOC_SCRATCH_BYTES (24u << 20)
qed_status qed_emit_noalloc(qed_tables tables, const qed_leptons *leptons, const qed_fields *fields,
                            const qed_step_params *params, const qed_photons *photons,
                            qed_counters *d_counters, qed_stream stream);

/* NBW step for photons [0, *d_count_prev): x += khat dt, fields at t + dt; pairs appended to
   `electrons` and `positrons` (same index in both for one pair); decayed photons become dead
   slots; survivors get the no-pair update.  Photons below k_retire are retired (dead slot).
   Sets *d_count_prev = *d_count on completion. */
qed_status qed_pair(qed_tables tables, const qed_photons *photons, const qed_fields *fields,
                    const qed_step_params *params, const qed_leptons *electrons,
                    const qed_leptons *positrons, qed_counters *d_counters, void *workspace,
                    size_t workspace_bytes, qed_stream stream);

/* Order-preserving removal of dead photon slots (id == 0); updates *d_count and
   *d_count_prev.  The workspace must hold qed_workspace_size(capacity) bytes plus a staging
   buffer of min(capacity, 2^26) photon records (the survivors are copied in rounds of that
   many): see qed_compact_workspace_size. */
size_t qed_compact_workspace_size(const qed_photons *photons, qed_precision precision);
qed_status qed_compact(const qed_photons *photons, qed_precision precision, void *workspace,
                       size_t workspace_bytes, qed_stream stream);

/* *d_clock += 1 on the stream (one-thread kernel), for replayed step sequences. */
qed_status qed_clock_advance(int64_t *d_clock, qed_stream stream);

/* Kernel timing for measurement tools: qed_profile_start clears the record and gives every
   subsequent launch a start and a stop event that the dispatch itself stamps (the kernel's begin
   and end, as a kernel trace reports them); qed_profile_stop synchronizes on them, writes
   up to max_entries per-kernel totals and the number of kernels seen, and stops recording.
   Process-wide and not thread-safe. */
qed_status qed_profile_start(void);
qed_status qed_profile_stop(qed_kernel_time *out, int max_entries, int *n_entries);

/* ---------------------------------------------------------------------------------------
   Whole steps of one or many independent instances (collisions) in three launches.

   One step of an instance is the paper's per-step sequence (NLC section flow chart for the
   leptons, NBW section for the photons): qed_emit for the electrons, qed_emit for the
   positrons, qed_pair for the photons stored before the step, then the step clock advances.
   qed_plan_step produces the same particles, bit for bit, for every instance at once: a lepton
   and a photon streaming launch over all particle sets (each set owns a contiguous range of
   blocks), then one launch that does the bookkeeping and processes the emitters and the
   decaying photons (with a learned inverse CDF too: the network runs in that launch); an
   instance with grid fields adds one launch that refreshes the plan's interleaved copy of its
   grid.  Appends keep the per-species order (photons of electrons, then of positrons, in
   emitter order; pairs in photon order). */
typedef struct {
    qed_leptons     electrons;   /* species 0 */
    qed_leptons     positrons;   /* species 1; stepped (and filled by pairs) only with QED_PAIR */
    qed_photons     photons;     /* filled with QED_EMIT; stepped with QED_PAIR */
    qed_fields      fields;
    qed_step_params params;      /* step and t at clock 0; d_clock is required: each
                                    qed_plan_step uses step + *d_clock, t + *d_clock dt and
                                    then adds 1 to *d_clock */
    qed_counters   *d_counters;  /* device, accumulated per instance */
} qed_instance;

typedef struct qed_surrogate_s *qed_surrogate;   /* opaque, library-owned; see below */

typedef struct {
    int particles_per_block;     /* blocks of a set = ceil(capacity / this), default 256 */
    int max_blocks_per_set;      /* cap on the blocks of one set; default: the blocks of the photon
                                    streaming kernel resident at once on the device (1024 on
                                    MI355X in single precision) */
    qed_surrogate icdf_nlc;      /* learned inverse CDF for the emission energy (NULL: tables); */
    qed_surrogate icdf_nbw;      /* ... for the pair split.  Only with QED_F32 tables, and built on
                                    the same tables (else QED_ERR_UNSUPPORTED / QED_ERR_INVALID).
                                    The network runs inside the processing launch, on the
                                    matrix cores, for the transitions each block holds; in the
                                    cells its last qed_surrogate_judge marked, the table inverse
                                    CDF is used. */
    int process_group;           /* streaming blocks whose transitions one block processes, default 4 */
    int photon_variant;          /* launch variant of the photon streaming pass (single precision, plain
                                    and plane-wave fields; ignored otherwise): 0 (default) tiles of
                                    1024 slots at four waves per SIMD, 1 tiles of 512 slots, 2 tiles of
                                    1024 at three waves per SIMD with the next tile's reads issued
                                    during the current tile's QED part; QED_ERR_INVALID outside 0..2.
                                    The results do not depend on it. */
} qed_plan_config;

typedef struct qed_plan_s *qed_plan;   /* opaque, library-owned */

/* Copy the instance descriptions (pointers, capacities, fields, parameters) to the device and
   allocate the plan's scratch: two mask planes of one bit per particle slot, per-block counts,
   per-set bookkeeping, per instance with grid fields 32 bytes per grid node and, per lepton set
   with QED_SUBCYCLE, 4 bytes per slot, 16 x 6 values of the tables' precision per slot (the
   momenta and P-vectors of the photons of a slot's sub-steps: 384 bytes in single, 768 in double
   precision) and 64 bytes per streaming block.  Allocates device memory
   and synchronizes the device; afterwards the arrays and counters named here must stay
   allocated and keep their addresses.  config may be NULL.  QED_ERR_INVALID for a NULL pointer,
   an inconsistent set (species, missing arrays, dt or eps_r <= 0, no d_clock or d_counters),
   QED_SUBCYCLE with QED_REJECTION or QED_OPTICAL_DEPTH, QED_REJECTION with QED_OPTICAL_DEPTH, or
   more than 2^24 blocks. */
qed_status qed_plan_create(qed_tables tables, int n_instances, const qed_instance *instances,
                           const qed_plan_config *config, qed_plan *out);

/* One step of every instance, enqueued on the stream without host synchronization; no
   allocation, no memset, so it can be captured in a HIP graph and replayed.  Steps of one plan
   must not overlap (they share its scratch). */
qed_status qed_plan_step(qed_plan plan, qed_stream stream);

/* Blocks in the plan's grid (0 for NULL). */
int64_t qed_plan_blocks(qed_plan plan);

/* Synchronize the device and release the plan.  Safe on NULL. */
qed_status qed_plan_destroy(qed_plan plan);

/* ---------------------------------------------------------------------------------------
   Learned inverse CDF.  The NLCS and NBW implementation sections tabulate the inverse CDF of
   the photon (pair) energy only for the two spin (xi3) channels, because the full dependence
   is too large to tabulate.  A surrogate stands in for the two fine tables of one process with
   nu(ln chi, rho, c) = base(ln chi, rho, c) + s y(u, v, c), c = -1 / +1 (NLC: spin down / up;
   NBW: xi3 = -1 / +1), s = 1.25 times the coarse table's largest error over 8 x 8 points per
   coarse cell (so that y spans about [-1, 1]; qed_surrogate_norm):
   - base: a coarse FP32 table of nu (the fine tables' values at its nodes; at least 4 ln chi
     nodes per decade over the fine table's range, rho nodes every 1 on [-20, 20]; 4-point
     Lagrange in each axis);
   - y: a network with inputs u = (ln chi - m)/h (m, h: centre and half-width of the table's
     ln chi range), v = rho/17 (rho = ln(r/(1-r)) of a 24-bit uniform, |rho| <= 16.64) and c;
     four hidden layers of 64 SiLU units and one linear output.  12801 parameters in the flat
     order W1 (3x64, row = input), b1, W2 (64x64, row = input unit), b2, W3, b3, W4, b4, W5 (64),
     b5.  The 64x64 layers run on the matrix cores in BF16 with FP32 accumulation (BF16 weights).
   The fine tables are the judge and the fallback: qed_surrogate_judge marks the coarse cells
   where the surrogate's error exceeds a bound, and there the table inverse CDF is used. */
int64_t qed_surrogate_n_params(void);

/* Allocate a surrogate for process 0 (NLC) or 1 (NBW) of these tables, parameters initialized
   from Philox channel 7 with `seed` (uniform, variance 2 / fan-in).  Synchronizes the device. */
qed_status qed_surrogate_create(qed_tables tables, int process, uint64_t seed, qed_surrogate *out);

/* Normalization constants {m, h, rho scale, residual scale} (host array of 4). */
qed_status qed_surrogate_norm(qed_surrogate s, float *out4);

/* Shape, judgement and size of a surrogate. */
typedef struct {
    int     process;
    int     n_params;
    float   in_m, in_h, rho_s, out_s;          /* as qed_surrogate_norm */
    float   base_lnchi0, base_dlnchi;          /* coarse ln chi nodes: base_lnchi0 + i base_dlnchi */
    int     base_n_chi;
    float   base_rho0, base_drho;              /* coarse rho nodes */
    int     base_n_rho;
    int64_t n_cells;                           /* 2 (base_n_chi - 1)(base_n_rho - 1): cell (c i j) */
    int64_t n_masked;                          /* cells marked by the last judgement */
    float   bound;                             /* its bound (0 before the first) */
    int64_t bytes_network, bytes_base, bytes_mask;  /* BF16 parameters, FP32 coarse table, mask */
} qed_surrogate_info;
qed_status qed_surrogate_get_info(qed_surrogate s, qed_surrogate_info *out);

/* `steps` Adam steps (lr; betas 0.9, 0.999) on the mean squared error of y against the residual
   (nu - base)/s, each on 4 x 256 x tiles_per_wave x 16 fresh samples drawn from Philox
   channel 6: ln chi uniform over the table range, rho half the time uniform over [-17, 17] and
   half the time logit(r) of a uniform r (as in the sampling), c = +-1; targets nu from the fine
   tables.  d_loss (device, `steps` floats, may be NULL) receives each step's mean squared
   error. */
qed_status qed_surrogate_train(qed_surrogate s, int steps, int tiles_per_wave, float lr, float *d_loss,
                               qed_stream stream);

/* Gradient of sum_i (y(x_i) - y_i)^2 over n given samples (device: d_x[n][3] = ln chi, rho, c;
   d_y[n]: targets of the network output) with respect to the parameters: d_grad[12801], then the
   sum of squares in d_grad[12801].  n <= 16384.  For checks of the training kernels. */
qed_status qed_surrogate_gradient(qed_surrogate s, const float *d_x, const float *d_y, int64_t n,
                                  float *d_grad, qed_stream stream);

/* nu for n samples d_x[n][3] = (ln chi, rho, c) (device) into d_nu[n]:
   QED_SURROGATE_AS_USED as the step uses it (the fine table in marked cells, else base + net),
   QED_SURROGATE_NETWORK base + net everywhere, QED_SURROGATE_BASE the coarse table alone. */
enum { QED_SURROGATE_AS_USED = 0, QED_SURROGATE_NETWORK = 1, QED_SURROGATE_BASE = 2 };
qed_status qed_surrogate_eval(qed_surrogate s, const float *d_x, int64_t n, int mode, float *d_nu,
                              qed_stream stream);

/* Judge the surrogate by the fine tables: for every coarse cell, the largest |base + net - table|
   over the centres of a points_per_axis^2 subdivision with |rho| <= 16.64 (cells beyond that
   rho are never reached by 24-bit uniforms and report 0), into cell_err (host, n_cells floats,
   may be NULL); cells above `bound` are marked, and the step and QED_SURROGATE_AS_USED use the
   table inverse CDF there.  *n_masked (may be NULL) receives their number.  Synchronizes the
   stream.  qed_surrogate_train and qed_surrogate_set_params clear the marks (a judgement holds
   for the parameters it saw): judge again after them. */
qed_status qed_surrogate_judge(qed_surrogate s, float bound, int points_per_axis, float *cell_err,
                               int64_t *n_masked, qed_stream stream);

/* Copy the FP32 parameters out of / into the surrogate (device arrays of 12801 floats). */
qed_status qed_surrogate_get_params(qed_surrogate s, float *d_params, qed_stream stream);
qed_status qed_surrogate_set_params(qed_surrogate s, const float *d_params, qed_stream stream);

/* Synchronize the device and release the surrogate.  Safe on NULL. */
qed_status qed_surrogate_destroy(qed_surrogate s);

#ifdef __cplusplus
}
#endif
#endif
