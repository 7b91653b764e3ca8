/*
 * nuosc -- bulb-model neutrino flavor evolution on MI355X (gfx950).
 *
 * C ABI of the library libnuosc.so.  No C++ types cross this boundary and no
 * exception escapes it.  Every call returns a nuosc_status; the message of the
 * last failure on a handle is available from nuosc_last_error().
 *
 * The problem is the one stated in Noormofidi, arXiv 1907.05560:
 *   - flavor wavefunction of n = 2 or 3 complex amplitudes per beam (eq 3.1),
 *     evolved by the Schrodinger equation i dpsi/dl = (H0 + Hm + Hnunu) psi
 *     (eq 3.2, eq 3.4 for the two-flavor form and the antineutrino map);
 *   - bulb geometry: along the trajectory emitted at cos(theta_0) = u the
 *     propagation cosine at radius r is c(r) = sqrt(1 - (R/r)^2 (1 - u^2))
 *     (eq 3.14) and dl = dr / c (eq 3.3);
 *   - neutrino self-interaction of the multi-angle bulb model (eq 3.8, 3.13,
 *     3.15) or of the single-angle model (eq 3.16-3.17);
 *   - Fermi-Dirac spectra (eq 4.1-4.2), vacuum term Delta = dm2 / 2E (eq 3.5-
 *     3.6), matter potential (eq 3.7) given as lambda(r) = lambda0 (rref/r)^p;
 *   - adaptive radial stepping with a global maximum error (Section 4.2.3) or
 *     a fixed step.
 *
 * Beams.  A beam is (species s, trajectory j, energy bin k) with s = 0 for
 * neutrinos born as nu_e and s = 1 for antineutrinos born as nubar_e; nu_x
 * and nubar_x enter through the spectral weights.  The beam index is
 *     b = (s * NA + j) * NE + k,      NA = max(n_angle, 1) * max(n_azimuth, 1),
 * and the number of beams is NB = 2 * NE * NA.  Energy bins sit at the
 * midpoints of [e_min, e_max]; emission-angle bins at the midpoints of
 * cos(theta_0) in (0, 1].  In the extended bulb model (n_azimuth > 1, eq
 * 3.18) trajectory j is emission-angle bin j / n_azimuth and azimuth bin
 * j % n_azimuth, azimuth bins at the midpoints of [0, 2 pi) sharing the
 * emission-angle weight equally.
 *
 * Frame.  Amplitudes are held in the frame co-rotating with the flavor-
 * diagonal part of the matter and self-interaction Hamiltonian of each
 * trajectory: psi = exp(-i sigma Phi_j) psi~ with sigma = +1 (nu), -1 (nubar)
 * and an FP64 phase Phi_j (n components) per trajectory.  Probabilities
 * |psi_a|^2 are the same in both frames.  NUOSC_FRAME_LAB keeps Phi = 0.
 *
 * Host state layout (nuosc_get_state / nuosc_set_state), always FP64:
 *     psi[a][2][NB]   component a, then re/im, then beam b;
 *     phase[NA][n]    co-rotating phase of trajectory j, component a.
 *
 * Units: r in km, Hamiltonians in km^-1, energies in MeV, dm2 in eV^2.
 *
 * Threading.  A handle is not thread-safe.  Distinct handles on distinct
 * streams are independent.  All work of a handle is ordered on its stream.
 */
#ifndef NUOSC_H
#define NUOSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NUOSC_OK = 0,
    NUOSC_E_INVALID = -1,       /* invalid argument or parameter set */
    NUOSC_E_NOMEM = -2,         /* device or host allocation failed */
    NUOSC_E_DEVICE = -3,        /* a HIP runtime call failed */
    NUOSC_E_NONFINITE = -4,     /* the step error became NaN or infinite */
    NUOSC_E_STEP_UNDERFLOW = -5,/* adaptive step fell below 1e-14 r */
    NUOSC_E_LIMIT = -6,         /* max_steps or max_wall_s reached */
    NUOSC_E_BUSY = -7           /* batch has no free slot or memory */
} nuosc_status;

/* Integrators.
 *   NUOSC_RK4_FIXED    classic RK4, n_fixed_steps equal steps.
 *   NUOSC_RK_DP54      adaptive embedded Dormand-Prince 5(4), max-norm error.
 *   NUOSC_EXP_STEPPER  the paper's own stepper: exponential steps
 *                      psi <- exp(-i H dl) psi (eq 3.10-3.12) inside its
 *                      half-step / full-step loop with averaging and a
 *                      maximum-error step control (Sections 4.2.3 and 5).
 *                      Lab frame, FP64, the bulb model (n_azimuth <= 1), one
 *                      run per handle (not in batches).  Per attempt: three
 *                      beam launches and three reduction launches; an
 *                      accepted attempt advances to the two-half-step estimate,
 *                      the error is its max-norm distance to the full-step one. */
enum { NUOSC_RK4_FIXED = 0, NUOSC_RK_DP54 = 1, NUOSC_EXP_STEPPER = 2 };
/* Precision of a run.
 *   NUOSC_FP64                amplitudes stored and advanced in FP64.
 *   NUOSC_FP32_AMP            amplitudes stored in FP32 and advanced with FP32
 *                             arithmetic (the per-beam state update), renormalised
 *                             at every accepted step; the update coefficients,
 *                             moments, step error, co-rotating phases and step
 *                             control in FP64.
 *   NUOSC_FP32_AMP_FP64_MATH  amplitudes stored in FP32 (renormalised every
 *                             step), the state update in FP64 registers. */
enum { NUOSC_FP64 = 0, NUOSC_FP32_AMP = 1, NUOSC_FP32_AMP_FP64_MATH = 2 };
enum { NUOSC_FRAME_COROTATING = 0, NUOSC_FRAME_LAB = 1 };

/* Parameters of one run.  Field names follow the configuration keywords of the
 * paper's Appendix A.3 (given in brackets). */
typedef struct nuosc_params {
    int32_t n_flavors;             /* [Flvs] 2 or 3 */
    int32_t n_energy;              /* [Ebins] >= 1 */
    double  e_min_mev, e_max_mev;  /* [E0] [E1] energy range, 0 <= e_min < e_max */
    int32_t n_angle;               /* [Abins] emission angles; 0 => single-angle model */
    double  lum_erg_s[4];          /* [Lve Lv_e Lvt Lv_t] nu_e, nubar_e, nu_x, nubar_x */
    double  mean_e_mev[4];         /* mean energies <E> of the same four species */
    double  eta[4];                /* [eta_ve ...] degeneracy parameters */
    double  dm2_ev2, theta;        /* [dm2] [theta] two flavors; dm2 < 0 = inverted */
    double  dm2_21_ev2, dm2_31_ev2;/* three flavors (PDG); dm2_31 < 0 = inverted */
    double  theta12, theta13, theta23, delta_cp;
    double  lambda0_km;            /* matter potential lambda(r) = lambda0 (rref/r)^p */
    double  lambda_rref_km;
    double  lambda_power;
    double  mu0_km;                /* self-interaction strength at the neutrinosphere */
    double  r_nu_km;               /* [Rv] neutrinosphere radius R */
    double  r_start_km, r_end_km;  /* [R0] [Rn], R <= r_start < r_end */
    int32_t integrator;            /* NUOSC_RK4_FIXED, NUOSC_RK_DP54 or NUOSC_EXP_STEPPER */
    int64_t n_fixed_steps;         /* RK4: equal steps from r_start to r_end */
    double  rtol;                  /* [eps0] adaptive integrators: max-norm error tolerance */
    double  dr_init_km;            /* [dr] first adaptive step */
    double  dr_max_km;             /* [max_dr] step cap */
    double  safety;                /* [ksi] controller safety factor in (0, 1] */
    int64_t max_steps;             /* [Ts] attempted-step limit, 0 = none */
    double  max_wall_s;            /* [Tn] wall-clock limit of one evolve call, 0 = none */
    int32_t precision;             /* NUOSC_FP64, NUOSC_FP32_AMP or NUOSC_FP32_AMP_FP64_MATH */
    int32_t frame;                 /* NUOSC_FRAME_COROTATING (default) or NUOSC_FRAME_LAB */
    int32_t n_azimuth;             /* azimuth bins per emission angle: the extended bulb
                                      model (eq 3.18, needs n_angle >= 1); 0 or 1 = bulb model */
} nuosc_params;

typedef struct nuosc_handle nuosc_handle;

/* Fill *p with the two-flavor single-angle defaults (1e51 erg/s, <E> 11/16/25
 * MeV, eta 0, dm2 -2.4e-3 eV^2, theta 0.1, lambda0 1e4 km^-1 (10 km/r)^3,
 * mu0 1e5 km^-1, R 10 km, 10 -> 250 km, RK4 with 1e4 steps, FP64). */
void nuosc_default_params(nuosc_params* p);

/* Device bytes nuosc_create needs for these parameters (state buffers,
 * tables, reduction scratch).  Returns 0 for an invalid parameter set. */
size_t nuosc_footprint_bytes(const nuosc_params* p);

/* Create a run in its initial state (every beam in its birth flavor at
 * r_start, phases zero).
 *   hip_stream        hipStream_t to order all work on, borrowed; NULL =>
 *                     the library creates and owns a stream.
 *   device_workspace  optional device memory of at least
 *                     nuosc_footprint_bytes(p) bytes owned by the caller and
 *                     kept alive until nuosc_destroy; NULL => the library
 *                     allocates and owns its buffers.
 * On failure *out is NULL and nothing is leaked. */
nuosc_status nuosc_create(const nuosc_params* p, void* hip_stream,
                          void* device_workspace, size_t workspace_bytes,
                          nuosc_handle** out);

/* Create a run in library-owned static device memory, allocating nothing:
 * for callers that cannot allocate device memory (code that is being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc).
 * The run behaves exactly as one made by nuosc_create (every other call of
 * this header applies to it and gives bitwise the same results); only its
 * device memory differs: all of it (state buffers, tables, reduction scratch,
 * control block) lies in one array of NUOSC_STATIC_SCRATCH_BYTES per GPU
 * that the library holds from its load until the process ends.  No device
 * memory is allocated or freed, here or by nuosc_destroy.
 *   p           run parameters; nuosc_footprint_bytes(p) must not exceed
 *               NUOSC_STATIC_SCRATCH_BYTES (else NUOSC_E_INVALID, with the
 *               two sizes in the message).
 *   hip_stream  stream to order all work on, borrowed; NULL is the null
 *               (legacy default) stream.  It must belong to the current
 *               device, which the run lives on.
 * The array is shared by every static run on its device and keeps the last
 * run's contents (creation rewrites all of it that a run reads before
 * writing): at most one static run per device is alive at a time, a second
 * nuosc_create_static on the same device returns NUOSC_E_BUSY until the
 * first is passed to nuosc_destroy.  Work on it from another process or
 * library copy does not share the array.  Synchronises the stream. */
#define NUOSC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
nuosc_status nuosc_create_static(const nuosc_params* p, void* hip_stream, nuosc_handle** out);

/* Make n_attempts step attempts (accepted or rejected; RK4 steps are always
 * accepted).  Attempts after the run reached r_end do nothing.  *n_accepted
 * (nullable) receives the number accepted by this call.  Returns
 * NUOSC_E_NONFINITE / NUOSC_E_STEP_UNDERFLOW when the run stopped on that
 * condition (state left at the last accepted step) and NUOSC_E_LIMIT when
 * max_steps was reached.  Synchronises the stream before returning.
 * Attempts in groups of 32 replay a HIP graph of 32 attempts, captured on the
 * run's stream at the first such call and owned by the handle (released by
 * nuosc_destroy); the rest, and every attempt while kernel timing is on, on
 * a run made by nuosc_create_static or on a stream that cannot be captured,
 * are launched directly.  The same holds for nuosc_evolve.  Not to be called
 * while the stream is being captured (it synchronises). */
nuosc_status nuosc_step(nuosc_handle* h, int64_t n_attempts, int64_t* n_accepted);

/* Queue n_attempts step attempts on the stream without waiting and without
 * reading back any status (for timing loops and graph replay): launched
 * directly, so that a caller may capture them.  The status is picked up by
 * the next nuosc_step / nuosc_stats call. */
nuosc_status nuosc_enqueue_steps(nuosc_handle* h, int64_t n_attempts);

/* Queue one launch of the current attempt: stage in 1..S with
 * S = nuosc_num_stages(h).  Runge-Kutta integrators (S = stages + 2: 6 for
 * RK4, 9 for Dormand-Prince): launches 1..S-2 complete the stages per
 * trajectory (launch S-2 also writes the coefficient tables of the update
 * and of the error), launch S-1 forms the new state and its step error
 * (beam pass), launch S runs the step control and, for an accepted attempt,
 * takes the power moments of the new state (beam pass).  Exponential
 * stepper (S = 3): every launch is a beam kernel followed by a reduction
 * kernel (the second timing interval below), the last one running the
 * controller.  A full attempt is launches 1..S in order; nuosc_enqueue_steps
 * does exactly that.  For timing tools that bracket individual kernels with
 * events.  NUOSC_E_INVALID for a stage out of range. */
nuosc_status nuosc_enqueue_stage(nuosc_handle* h, int32_t stage);

/* Number of launches S of one step attempt. */
int32_t nuosc_num_stages(const nuosc_handle* h);

/* Kernel timing for measurement tools.  While enabled, every launch records
 * HIP events on the handle's stream before its main kernel, after it, and
 * after its second kernel (the moment launch 0 and every launch of the
 * exponential stepper have one; the second interval is empty for the
 * others).
 * nuosc_timing_read waits for the stream, adds the elapsed times of all
 * launches recorded since the last read into per-stage sums and writes them:
 * beam_ms and fin_ms (milliseconds, nuosc_num_stages(h) + 1 entries each,
 * index = stage, 0 being the moment launch of create / set_state / moments;
 * fin_ms holds the second interval) and count (launches per stage, same
 * length); each pointer nullable.  The sums are cleared by the read.
 * Enabling or disabling clears them too.  Timing adds three event records
 * per launch (a few microseconds each on the stream) and changes no
 * result. */
nuosc_status nuosc_timing_enable(nuosc_handle* h, int32_t on);
nuosc_status nuosc_timing_read(nuosc_handle* h, double* beam_ms, double* fin_ms, int64_t* count);

/* Evolve until r = min(r_target, r_end) (the last step is clipped to land on
 * it), or until max_steps / max_wall_s is reached (NUOSC_E_LIMIT). */
nuosc_status nuosc_evolve(nuosc_handle* h, double r_target_km);

/* Angle moments of the current state at the current radius:
 *   J0 = sum_j w_j S_j,  J1 = sum_j w_j c_j S_j  (multi-angle, eq 3.13-3.15)
 *   J0 = D(r/R) S_0,     J1 = 0                  (single angle, eq 3.16-3.17)
 * with S_j = sum_k [g_k rho(nu) - gbar_k conj(rho(nubar))], rho = 2 psi psi^+
 * in the lab frame.  j0, j1: n*n complex each, row-major, interleaved re/im
 * (host memory, written).  r_km (nullable) receives the radius. */
nuosc_status nuosc_moments(nuosc_handle* h, double* j0, double* j1, double* r_km);

/* The extended model's azimuth moments of the current state (eq 3.18):
 *   J2 = sum_j w_j s_j cos(phi_j) S_j,  J3 = sum_j w_j s_j sin(phi_j) S_j,
 * s_j = sin(theta_j); zero for the bulb model.  Layout as nuosc_moments. */
nuosc_status nuosc_moments_azimuth(nuosc_handle* h, double* j2, double* j3);

/* Survival probabilities P_b = |psi_b,1|^2 of every beam (host, NB doubles). */
nuosc_status nuosc_probabilities(nuosc_handle* h, double* p_out);

/* Checkpoint: copy the state to / from host buffers laid out as described
 * above (psi: n*2*NB doubles, phase: NA*n doubles).  set_state also sets the
 * radius and the next adaptive step, resets the step counters and recomputes
 * the moments of the new state.  In FP32_AMP runs the amplitudes are stored
 * in FP32 (set_state rounds them). */
nuosc_status nuosc_get_state(nuosc_handle* h, double* psi, double* phase);
nuosc_status nuosc_set_state(nuosc_handle* h, const double* psi, const double* phase,
                             double r_km, double dr_km);

/* Energy-averaged flavor content of every trajectory: the paper's second
 * dump mode (Section 4.2.4, the average flavor state over the energy bins of
 * one trajectory), computed on the device from the current state:
 *   out[s][j][a] = sum_k f_sk |psi_{s,j,k,a}|^2 / sum_k f_sk
 * for species s (0 neutrino, 1 antineutrino), trajectory j < NA and flavor
 * a < n, with f_sk the number flux of the species' birth flavor (nu_e or
 * nubar_e, eq 4.1-4.2) in energy bin k; the plain mean over bins if it sums
 * to zero.  out: host, 2*NA*n doubles, written before the call returns. */
nuosc_status nuosc_energy_average(nuosc_handle* h, double* out);

/* The same average queued on the handle's stream into device memory
 * out_device (2*NA*n doubles, owned by the caller), without waiting: for
 * callers that keep the result on the device and for timing. */
nuosc_status nuosc_enqueue_energy_average(nuosc_handle* h, double* out_device);

/* Snapshots: the paper's first dump mode and resume (Section 4.2.4).  A
 * snapshot file holds this header, then the state in the host layout above
 * (psi: n*2*NB doubles, phase: NA*n doubles), then a 64-bit FNV-1a hash of
 * all preceding bytes; integers and doubles are little-endian as in memory:
 *   "NUOSCSN1" (8 bytes), nuosc_snapshot_header (72 bytes), payload, hash.
 * nuosc_snapshot_write stores the current state, radius, next step, step
 * counters and the controller's rejection flag.  nuosc_snapshot_read restores them into a run with the same
 * flavors, energy and angle grid and frame (as nuosc_set_state, then the
 * counters and the flag); the precision may differ (FP32 runs round the amplitudes).
 * nuosc_snapshot_info reads and checks a file's header and hash without a
 * handle.  A missing, truncated or corrupted file, or a grid mismatch, gives
 * NUOSC_E_INVALID and leaves the run unchanged. */
typedef struct {
    int32_t n_flavors, n_energy, n_angle;   /* as in nuosc_params */
    int32_t precision, integrator, frame;
    int32_t last_rejected;                  /* the last attempt was rejected (no step growth next) */
    int32_t reserved;                       /* 0 */
    int64_t n_beams;                        /* NB */
    double  r_km, dr_km;                    /* radius of the state, next step */
    int64_t accepted, rejected;             /* step counters */
} nuosc_snapshot_header;

nuosc_status nuosc_snapshot_write(nuosc_handle* h, const char* path);
nuosc_status nuosc_snapshot_read(nuosc_handle* h, const char* path);
nuosc_status nuosc_snapshot_info(const char* path, nuosc_snapshot_header* info);

/* Step statistics (each pointer nullable). */
nuosc_status nuosc_stats(nuosc_handle* h, int64_t* accepted, int64_t* rejected,
                         double* r_km, double* dr_km);

/* Number of beams NB and trajectories NA of the run. */
int64_t nuosc_num_beams(const nuosc_handle* h);
int32_t nuosc_num_traj(const nuosc_handle* h);

/* Message of the last failure on h (or of the last failed create when h is
 * NULL); valid until the next call on the same handle. */
const char* nuosc_last_error(const nuosc_handle* h);

/* Release the handle and everything it owns.  NULL-safe. */
void nuosc_destroy(nuosc_handle* h);

/* ---------------------------------------------------------------- batches
 * Continuous batching of independent runs (the serving pattern): runs with
 * different grids, spectra, luminosities and mixing parameters are admitted
 * into slots while others are being stepped, keep their state resident in
 * device memory, and are advanced together -- every launch of a batch step
 * covers all active runs, each workgroup belonging to exactly one run, so a
 * run's result is bitwise the same alone and in any mix.  All runs of a batch
 * share n_flavors, precision and integrator.  Device memory for the runs
 * comes from one arena; admission fails with NUOSC_E_BUSY when no slot is
 * free or the arena has no gap of nuosc_footprint_bytes(p) bytes. */
typedef struct nuosc_batch nuosc_batch;

/* Create a batch of at most max_slots runs (1..1024).
 *   hbm_budget_bytes  size of the device arena the runs are placed in
 *   hip_stream        stream to order all work on, borrowed; NULL => own stream
 *   device_arena      optional caller-owned device memory of hbm_budget_bytes
 *                     (kept alive until nuosc_batch_destroy); NULL => allocated
 * integrator is NUOSC_RK4_FIXED or NUOSC_RK_DP54 (the exponential stepper runs
 * as single runs only).  NUOSC_E_INVALID for bad arguments, NUOSC_E_NOMEM when
 * the arena cannot be allocated.  On failure *out is NULL. */
nuosc_status nuosc_batch_create(int32_t max_slots, int32_t n_flavors, int32_t precision, int32_t integrator,
                                size_t hbm_budget_bytes, void* hip_stream, void* device_arena,
                                nuosc_batch** out);

/* Admit a run in its initial state; *slot receives its slot.  NUOSC_E_BUSY:
 * no free slot or no arena gap large enough (nothing changes); NUOSC_E_INVALID:
 * invalid parameters, n_flavors / precision / integrator differ from the
 * batch's, or the run is an extended-model run (n_azimuth > 1: batches serve
 * the bulb model).  Synchronises the stream. */
nuosc_status nuosc_batch_admit(nuosc_batch* b, const nuosc_params* p, int32_t* slot);

/* Make n_attempts step attempts of every admitted run that is still running
 * (when the same set of runs is stepped with the same count twice in a row,
 * the launch sequence is captured as a HIP graph and replayed from then on).  *n_finished (nullable) receives the
 * number of admitted runs that have stopped (reached r_end, or stopped on an
 * error or limit).  Synchronises the stream. */
nuosc_status nuosc_batch_step(nuosc_batch* b, int64_t n_attempts, int32_t* n_finished);

/* State of the run in a slot (each pointer nullable): accepted and rejected
 * steps, radius, and its status (NUOSC_OK while running or after reaching
 * r_end, which *done reports as 1; else the error it stopped on). */
nuosc_status nuosc_batch_query(nuosc_batch* b, int32_t slot, int64_t* accepted, int64_t* rejected,
                               double* r_km, int32_t* done, int32_t* run_status);

/* Number of beams of the run in a slot (0 for a free slot). */
int64_t nuosc_batch_num_beams(const nuosc_batch* b, int32_t slot);

/* Remove the run in a slot, first writing its survival probabilities to
 * p_out (host, NB doubles; nullable), and free its memory and slot. */
nuosc_status nuosc_batch_retire(nuosc_batch* b, int32_t slot, double* p_out);

/* How the batch's steps ran (each pointer nullable): nuosc_batch_step calls
 * that launched work directly on the stream, calls that replayed the captured
 * graph, and how many graphs were captured (a capture is counted in the call
 * that replays it first). */
nuosc_status nuosc_batch_graph_stats(const nuosc_batch* b, int64_t* eager_steps, int64_t* graph_steps,
                                     int64_t* captures);

/* Number of occupied slots. */
int32_t nuosc_batch_occupied(const nuosc_batch* b);

/* Message of the last failure on b (or of the last failed batch create when
 * b is NULL). */
const char* nuosc_batch_last_error(const nuosc_batch* b);

/* Release the batch, its runs and everything it owns.  NULL-safe. */
void nuosc_batch_destroy(nuosc_batch* b);

#ifdef __cplusplus
}
#endif
#endif
