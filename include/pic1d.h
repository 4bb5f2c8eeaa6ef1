/*
 * pic1d.h -- C ABI of an MI355X (gfx950) implementation of the 1D3V electrostatic
 * PIC/MCC step for capacitively coupled RF discharges (Becker, Kaehlert, Sun, Bonitz,
 * Loffhagen, "Advanced fluid modelling and PIC/MCC simulations of low-pressure ccrf
 * discharges", arXiv:1608.04601).
 *
 * One step (Sec. 2.5): cloud-in-cell field gather, velocity-Verlet push, full absorption
 * at both electrodes, cloud-in-cell charge deposition, the Poisson equation (Sec. 2,
 * Eq. "poisson") with phi(0,t) = V0 sin(2 pi f t) and phi(d,t) = 0 (Sec. 2.2), and
 * null-collision Monte Carlo collisions for the processes of Table "tab:reactions".
 *
 * Conventions for every function:
 *   - units are SI, energies in eV;
 *   - every pointer argument is a HOST pointer unless its comment says otherwise;
 *     output arrays are owned by the caller, input arrays are copied before return;
 *   - functions return PIC_OK (0) or a negative PIC_E* status and never throw;
 *   - work is enqueued on one HIP stream (the caller's, or the library's own); device
 *     faults (capacity, non-finite values) are raised on the device and reported by
 *     the next synchronising call (pic_sync, pic_moments, pic_get_*); after any error
 *     the handle is poisoned: every later call returns that first error, and only
 *     pic_free and pic_last_error remain useful;
 *   - a handle must not be used from two threads at once.
 */
#ifndef PIC1D_H
#define PIC1D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PIC_OK          0
#define PIC_EINVAL     -1  /* invalid argument or configuration (checked on the host)       */
#define PIC_ENOMEM     -2  /* host or device allocation failed                              */
#define PIC_EHIP       -3  /* a HIP runtime call failed                                     */
#define PIC_ECAPACITY  -4  /* particle storage, per-step birth buffer or id space exhausted */
#define PIC_ENUMERIC   -5  /* a particle coordinate became non-finite                      */
#define PIC_ESTATE     -6  /* call not allowed in the handle's state                       */

/* ---- collision processes (Table "tab:reactions"; Sec. 2.5 scattering rules) ----
 * Electron processes see a gas atom at rest; ion processes see an atom drawn from the gas
 * Maxwellian at T_gas.  ELASTIC/ISOTROPIC scatter isotropically in the centre-of-mass
 * frame; EXCITATION removes the threshold energy and scatters isotropically; IONIZATION
 * shares the remaining energy equally between the two electrons (both isotropic) and
 * creates an ion from the gas Maxwellian at the parent's position; BACKWARD gives the
 * ion the atom's velocity (charge exchange). */
#define PIC_E_ELASTIC     0
#define PIC_E_EXCITATION  1
#define PIC_E_IONIZATION  2
#define PIC_I_ISOTROPIC   3
#define PIC_I_BACKWARD    4
/* energy frame of a table (Sec. 4.1: He ion data in centre-of-mass energy, Ar in lab) */
#define PIC_FRAME_LAB 0
#define PIC_FRAME_CM  1
#define PIC_MAX_PROCESSES 16
#define PIC_MAX_CELLS 4096
#define PIC_NOALLOC_MAX_POINTS 1024   /* profile points of pic_load_profiles_noalloc */

#define PIC_ELECTRON 0
#define PIC_ION      1

/* One cross-section table.  sigma(eps) = 0 for eps < threshold_eV; otherwise eps is
 * raised to emin_eV, then sigma is the last value at or beyond the last point and the
 * linear interpolation of sigma_m2[k] at eps_k = k * de_eV in between.  LAB tables are
 * read at 1/2 m_s g^2, CM tables at 1/2 mu g^2 (g: speed relative to the atom). */
typedef struct pic_xsec {
    int32_t kind;             /* PIC_E_* or PIC_I_*; the species follows from the kind */
    int32_t frame;            /* PIC_FRAME_LAB or PIC_FRAME_CM                          */
    int32_t n_points;         /* >= 2                                                   */
    int32_t reserved;         /* must be 0                                              */
    double threshold_eV;      /* >= 0                                                   */
    double de_eV;             /* > 0                                                    */
    double emin_eV;           /* >= 0; 0 = no floor (Sec. 4.1 uses 0.1 eV for Ar ions)   */
    const double* sigma_m2;   /* host, n_points finite values >= 0; copied by pic_init  */
} pic_xsec;

/* The problem statement (Sec. 2, Table "tab:discharge") and the numerical parameters
 * (Sec. 4.2, Table "tab:numericalparameters").  The superparticle weight is
 * W = n_init_m3 * gap_m / n_init_super[0] per m^2, the same for both species; the gas
 * density is pressure / (k_B T_gas) (Sec. 2.1); the ion mass is the gas mass. */
typedef struct pic_config {
    double gap_m;               /* electrode distance d > 0                            */
    double pressure_Pa;         /* > 0                                                 */
    double gas_temperature_K;   /* > 0                                                 */
    double gas_mass_amu;        /* > 0                                                 */
    double rf_voltage_V;        /* V0 at the powered electrode z = 0 (finite)          */
    double rf_frequency_Hz;     /* f > 0                                               */
    double dt_s;                /* time step > 0                                       */
    double n_init_m3;           /* initial uniform density >= 0                        */
    double te_init_eV;          /* k_B T of the initial electron Maxwellian, >= 0      */
    double ti_init_eV;          /* k_B T of the initial ion Maxwellian, >= 0           */
    int32_t n_cells;            /* 2 .. PIC_MAX_CELLS cells, n_cells + 1 nodes         */
    int32_t n_xsec;             /* 0 .. PIC_MAX_PROCESSES, at most 8 per species       */
    const pic_xsec* xsec;       /* host array of n_xsec tables, in selection order     */
    int64_t n_init_super[2];    /* initial particles per species; [0] > 0              */
    int64_t capacity[2];        /* storage per species, >= n_init_super, < 2^31        */
    uint64_t seed;              /* Philox key                                          */
    int32_t sort_every;         /* cell sort + compaction every this many steps; 0 = never */
    int32_t moments_every;      /* moment sample every this many steps, >= 1           */
    int32_t max_births_per_step;/* ionisations one step may create, >= 1               */
    int32_t launch_blocks;      /* workgroups of the particle pass; 0 = automatic      */
    int32_t electron_order;     /* periodic reordering of the electrons: 1 = sort by cell,
                                   0 = only remove absorbed slots (order kept), -1 = automatic:
                                   sort when a 3 eV thermal electron crosses at most 16 cells per
                                   sort interval.  Ions are always sorted by cell.  Results do
                                   not depend on this choice. */
    int32_t reserved;           /* must be 0                                           */
    double j0_target_A_m2;      /* 0: V0 stays rf_voltage_V.  > 0: current-driven operation
                                   (Sec. 2, Eq. "adaptivevoltage"): at the end of every whole RF
                                   period the amplitude becomes V0 J0 / J_calc, J_calc the
                                   period's max |J|; finite, >= 0 */
} pic_config;

/* Window averages since the last reset (pic_moments).  Arrays are caller-owned host
 * arrays of n_nodes = n_cells + 1 doubles, or NULL to skip.  Densities and the ion flux
 * divide the cloud-in-cell sums by the node volume (dx inside, dx/2 at the electrodes)
 * and the number of samples; the mean electron energy is the ratio of window sums
 * (U_e = w_e / n_e, Sec. 2.1), NaN where no electron was sampled. */
typedef struct pic_moments_out {
    int32_t n_nodes;            /* in: length of the arrays below                      */
    int32_t reserved;
    double* n_e_m3;
    double* n_i_m3;
    double* mean_energy_e_eV;
    double* phi_V;              /* window mean of the node potential                  */
    double* flux_i_m2s;         /* ion particle flux along z                           */
    int64_t n_samples;
    int64_t n_steps;            /* steps in the window                                 */
    double window_s;
    double J0_A_m2;             /* mean over whole RF periods of max |J| (Sec. 2.2)    */
    double flux_i_powered_m2s;  /* ions absorbed at z = 0 per area and time (Table "tab:plasmaparameters") */
    int64_t absorbed[2][2];     /* [species][electrode 0 = z=0, 1 = z=d] in the window */
} pic_moments_out;

/* Running counters (pic_get_counters). */
typedef struct pic_counters {
    int64_t step;                    /* completed steps n (state at t_n = n dt)        */
    int64_t n_alive[2];
    int64_t n_slots[2];              /* storage in use, including absorbed holes       */
    int64_t next_id[2];
    int64_t particle_steps;          /* sum over steps of the particles alive at its start */
    int64_t absorbed_total[2][2];
    int64_t collisions[PIC_MAX_PROCESSES]; /* real collisions per table, config order   */
    int64_t numax_violations[2];     /* candidates whose frequency exceeded nu_max      */
    int64_t births_total;
    double J_last_A_m2;              /* J^{n-1/2} of the last step (Sec. 2.2)            */
    double sigma0_C_m2;              /* surface charge eps0 E(0) on the powered electrode */
    double sigmad_C_m2;              /* surface charge -eps0 E(d) on the grounded one     */
    double V0_V;                     /* RF amplitude in use (changes only when current-driven) */
} pic_counters;

/* Constants the library derived from the configuration (pic_get_derived). */
typedef struct pic_derived {
    double dx_m;
    double n_gas_m3;
    double weight_m2;
    double ion_mass_kg;
    double v_thermal_gas_ms;         /* sqrt(k_B T_gas / M)                             */
    double numax_s[2];               /* null-collision bound per species                */
    double p_null[2];                /* 1 - exp(-numax dt)                               */
    uint32_t threshold[2];           /* candidate iff (philox word >> 8) < threshold    */
    int32_t steps_per_period;
    int32_t reserved;
} pic_derived;

typedef struct pic_handle pic_handle;

/* ---- the production entry points ---- */

/* Validate cfg, derive the constants, allocate device storage, load the uniform
 * Maxwellian initial state (Sec. 2.2) and solve the field at t = 0.  hip_stream is a
 * hipStream_t on the current device, or NULL for the device's null stream; all work of the
 * handle is ordered on it, and the caller keeps it alive until pic_free.  On error *out is
 * NULL and the status says why (pic_last_error(NULL) gives the message). */
int pic_init(const pic_config* cfg, void* hip_stream, pic_handle** out);

/* Enqueue n_steps >= 0 PIC/MCC steps (Sec. 2.5) on the handle's stream and return
 * without waiting.  The collisions of the last step complete lazily at the next step or
 * at the next call that reads the state.  With a graph size set (pic_set_graph), runs of
 * that many steps are replayed from a captured HIP graph (captured on first use and again
 * whenever the reordering phase or the pending state differs from the captured one); the
 * rest, and every step while pic_timing is on, are launched one by one.  Results do not
 * depend on which. */
int pic_step(pic_handle* h, int64_t n_steps);

/* Steps per captured graph for pic_step: 0 (the default) launches every step directly;
 * an RF period (1 / (f dt) steps, Sec. 2.2) replays one graph per period.  Must be in
 * [0, 100000] (PIC_EINVAL otherwise); waits for the stream and drops any captured graph.
 * The graph is captured on a private stream of default priority and launched on the
 * handle's stream; it holds kernel launches only.  pic_set_record_decisions drops it. */
int pic_set_graph(pic_handle* h, int64_t steps_per_graph);

/* Number of graph replays since the last pic_set_graph (for tests). */
int pic_graph_launches(const pic_handle* h, int64_t* n);

/* Launch shape of the particle pass, fixed at pic_init: workgroups, threads per workgroup,
 * and dynamic = 1 when the pass takes its slots in blocks from a per-species counter as
 * workgroups become free (chosen when every workgroup starts with at least 65536 slots;
 * otherwise 0: each workgroup has a fixed contiguous slot range).  Results do not depend on
 * it.  Any output pointer may be NULL; PIC_EINVAL if h is NULL. */
int pic_launch_shape(const pic_handle* h, int* blocks, int* threads, int* dynamic);

/* Wait for the handle's stream and report deferred device errors. */
int pic_sync(pic_handle* h);

/* Complete the pending step, synchronise, and write the window averages since the last
 * reset into *out (arrays sized out->n_nodes == n_cells + 1).  reset != 0 starts a new
 * window after reading. */
int pic_moments(pic_handle* h, pic_moments_out* out, int reset);

/* Release the handle and its device storage.  NULL-safe; waits for queued work. */
void pic_free(pic_handle* h);

/* Message of the last error on h (or of the last failed pic_init when h is NULL).
 * Valid until the next call on h. */
const char* pic_last_error(const pic_handle* h);

/* ---- inspection and test hooks ---- */

/* Complete the pending step, synchronise and read the running counters. */
int pic_get_counters(pic_handle* h, pic_counters* out);
int pic_get_derived(const pic_handle* h, pic_derived* out);

/* Copy the alive particles of one species (state at t_n, integer-time velocities) into
 * caller arrays of length capacity; *n_out receives the count.  Positions are metres in
 * double precision (the device keeps FP32 positions in cell units, whose value in metres
 * is exact in FP64); velocities are m/s.  If all array pointers are NULL only the count
 * is returned.  Returns PIC_EINVAL if capacity is too small. */
int pic_get_particles(pic_handle* h, int species, double* x, float* vx, float* vy, float* vz,
                      uint32_t* id, int64_t capacity, int64_t* n_out);

/* Replace the particles of one species (n <= capacity, 0 < x < d, finite velocities,
 * ids < next_id <= 2^32) and the step counter; the field is re-solved at t_step. */
int pic_set_particles(pic_handle* h, int species, const double* x, const float* vx, const float* vy,
                      const float* vz, const uint32_t* id, int64_t n, uint32_t next_id, int64_t step);

/* Node charge per area (C/m^2) deposited for the current field, node potential and node
 * field at t_n; arrays of n_cells + 1 values, NULL to skip. */
int pic_get_fields(pic_handle* h, double* q_nodes, double* phi, float* e_nodes);

/* Warm start: replace the initial load of a discharge that has not been stepped by one
 * drawn from cycle-averaged profiles given on n_points >= 2 equally spaced points spanning
 * [0, d] (both electrodes included), linear in between: electron and ion densities
 * [m^-3, >= 0], mean electron energy [eV, >= 0] and ion flux [m^-2 s^-1, along +x].
 * The periodic state does not depend on the initial state (Sec. 3, on initial values),
 * so the load only changes how long the discharge takes to reach it.
 * Species s gets N_s = round(integral n_s dx / W) particles (W the constant weight,
 * Sec. 2.5), positions by inverting the cumulative integral of the density, electrons
 * Maxwellian at k_B T_e = (2/3) <eps_e>(x), ions Maxwellian at the gas temperature with
 * mean v_x = Gamma_i / n_i (0 where n_i = 0), ids 0 .. N_s - 1, Philox counters
 * (k, 0, 0 and 1, (s << 8) | 0xFE).  Then deposits and solves the field at t = 0.
 * Host arrays, copied; synchronises.  PIC_ESTATE if the discharge was stepped,
 * PIC_ECAPACITY if N_s exceeds the capacity, PIC_EINVAL for bad profiles. */
int pic_load_profiles(pic_handle* h, int32_t n_points, const double* n_e, const double* n_i,
                      const double* mean_energy_e_eV, const double* flux_i);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pic_load_profiles with the same
 * arguments, results and errors, except that it allocates nothing.  Its staging table
 * lives in a fixed device array of the library, 2 x 4 x PIC_NOALLOC_MAX_POINTS doubles
 * (64 KiB) per GPU, held until the process ends; n_points above PIC_NOALLOC_MAX_POINTS is
 * rejected with PIC_EINVAL.  The handle's device must be current.  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU (from several host threads)
 * race; each call overwrites what it uses before reading it. */
int pic_load_profiles_noalloc(pic_handle* h, int32_t n_points, const double* n_e, const double* n_i,
                              const double* mean_energy_e_eV, const double* flux_i);

/* ---- Diagnostics of the results section (off the particle pass).  A diagnostic window
 * adds up samples of the completed electron state at chosen time levels: call
 * pic_diag_sample every k steps for time averages, or once per RF period at a fixed phase
 * (the paper's t f = 0.25) for phase-resolved profiles.  Per node (cloud-in-cell weights,
 * node volume dx, dx/2 at the electrodes, constant weight W, averaged over the samples):
 * n_e; U_e = w_e / n_e; the electron particle flux Gamma_e = sum v_x and energy flux
 * Q_e = sum e0 U v_x; the ionisation rate S = sum n_gas sigma_iz(U) |v| (the expected rate
 * of each electron on the ionisation tables); the density of fast electrons, U > |V0| / 4
 * with the amplitude in use; the heating rate -e0 E Gamma_e formed per sample; the field.
 * And the time and space averaged isotropic distribution f0(U)/n_e at the centres of
 * n_bins energy bins over [0, u_max): count_k / (N dU sqrt(U_k)) with N every sampled
 * electron, so that the integral of f0 sqrt(U) dU over all energies is n_e. */
typedef struct pic_diag_out {
    int32_t n_nodes;              /* in: n_cells + 1                                     */
    int32_t n_bins;               /* in: the configured bin count (when eedf is set)     */
    double* n_e_m3;               /* caller-owned [n_nodes] arrays, or NULL to skip      */
    double* mean_energy_e_eV;     /* NaN where no electron was sampled                   */
    double* flux_e_m2s;
    double* energy_flux_e_W_m2;
    double* ionisation_rate_m3s;
    double* n_fast_m3;
    double* heating_W_m3;
    double* E_V_m;
    double* eedf_eV_m32;          /* [n_bins] f0/n_e at the bin centres [eV^-3/2]        */
    int64_t n_samples;            /* out */
    int64_t n_electrons;          /* out: electrons summed over the samples              */
    double u_max_eV;              /* out */
} pic_diag_out;

/* Allocate (first call) and clear the diagnostic window with n_bins in [1, 4096] energy
 * bins over [0, u_max_eV).  6 (n_cells + 1) + n_bins words must fit 160 KiB of LDS. */
int pic_diag_config(pic_handle* h, int32_t n_bins, double u_max_eV);

/* Complete the pending step (as pic_sync does, without waiting) and add the state at the
 * current time level to the window; enqueued.  PIC_ESTATE before pic_diag_config. */
int pic_diag_sample(pic_handle* h);

/* Averages over the window's samples into *out (synchronises); reset clears the window. */
int pic_diag_read(pic_handle* h, pic_diag_out* out, int reset);

/* Electron and ion particle fluxes into the powered electrode (z = 0) against time over
 * the last RF period [m^-2 s^-1]: entry k is W N_k / dt with N_k the particles absorbed
 * there during the step that started at phase k / n of the period, from the most recent
 * period that reached that phase (recorded by every step).  n must be the steps per RF
 * period (pic_get_derived).  Synchronises. */
int pic_electrode_fluxes(pic_handle* h, int32_t n, double* gamma_e, double* gamma_i);

/* Record, for every collision test, the outcome per particle: 0 not a candidate,
 * 1 null collision, 2 + j table j selected.  Recording costs one byte per particle per
 * step and is off by default. */
int pic_set_record_decisions(pic_handle* h, int on);

/* Outcomes of the most recent collision test for the alive particles of one species. */
int pic_get_decisions(pic_handle* h, int species, uint32_t* id, int8_t* code, int64_t capacity,
                      int64_t* n_out);

/* Mean duration (ms) of the particle-pass kernel over the last timed window started by
 * pic_timing(h, 1) and read by pic_timing(h, 0); measured with HIP events on the
 * handle's stream.  *n_launches receives the number of timed launches. */
int pic_timing(pic_handle* h, int start, double* mean_ms, int64_t* n_launches);

/* ---- Batches of independent discharges (a parameter sweep, the paper's study design,
 * Table "tab:discharge": several pressures and gases) advanced together: one particle-pass
 * launch per step serves every discharge of the batch, each on its own share of the
 * workgroups (in proportion to its particles) and with its own field solve.  Results are
 * those of advancing each discharge alone (bitwise, per particle id). */
typedef struct pic_batch pic_batch;

/* Create n >= 1 discharges from cfgs[0..n-1] on one HIP stream (NULL = null stream).  All
 * must fit one workgroup size: either every n_cells <= 2047 or every n_cells > 1024.
 * launch_blocks of the configs is ignored for batched steps.  On error *out is NULL. */
int pic_batch_init(const pic_config* cfgs, int n, void* hip_stream, pic_batch** out);

/* Enqueue n steps of every discharge; returns without waiting.  Discharges left with
 * different pending states by per-discharge calls are first brought to the same state.
 * When every discharge is due for reordering in the same step, the reordering runs as one
 * launch per stage for all of them.  With a graph size set (pic_batch_set_graph), runs of
 * that many steps are replayed from a captured HIP graph (captured on first use and again
 * whenever the discharges' reordering phases differ from the captured ones); the rest, and
 * every step while timing is on, are launched one by one.  Results do not depend on which. */
int pic_batch_step(pic_batch* b, int64_t n_steps);

/* Steps per captured graph for pic_batch_step: 0 (the default) launches every step
 * directly; an RF period of the discharges (1 / (f dt) steps) replays one graph per
 * period.  Must be in [0, 100000]; waits for the stream and drops any captured graph.  The
 * graph is captured on a private stream of default priority and launched on the batch's
 * stream; it holds kernel launches only. */
int pic_batch_set_graph(pic_batch* b, int64_t steps_per_graph);

/* Completes every discharge's pending step, then splits the workgroups of batched launches
 * anew in proportion to the particles alive now (the split made at pic_batch_init follows
 * the initial counts, which a warm start or an ionising transient can change several-fold).
 * Drops any captured graph.  Results do not depend on the split. */
int pic_batch_rebalance(pic_batch* b);

/* Number of graph replays since the last pic_batch_set_graph (for tests). */
int pic_batch_graph_launches(const pic_batch* b, int64_t* n);

/* Test hook: pic_set_record_decisions for every discharge of the batch, so that batched
 * launches write the per-slot collision decisions that pic_get_decisions reads through
 * pic_batch_handle.  Completes pending steps and drops any captured graph; allocates the
 * records on first use. */
int pic_batch_set_record_decisions(pic_batch* b, int on);

/* Launch and reordering schedule chosen by pic_batch_autotune. */
typedef struct pic_tuning {
    int32_t threads;         /* workgroup size of the batched particle pass */
    int32_t sort_every;      /* steps between reorderings, every discharge */
    int32_t electron_order;  /* 1 electrons sorted by cell, 0 compacted in order, -1 each
                                discharge's own choice from pic_config.electron_order */
    int32_t trials;          /* configurations timed */
    double rounds;           /* workgroups per launch, in units of those resident at once */
    double ms_per_step;      /* measured mean time per batched step, reordering included */
} pic_tuning;

/* Picks the batched pass's workgroup size and launch size, the reordering interval and the
 * electron ordering by timing eager trials of about steps_per_trial steps (at least two
 * reordering intervals) on the batch itself, one coordinate at a time, and keeps the
 * fastest.  The trials advance every discharge; results do not depend on the choices, only
 * the time per step does.  Needs every discharge created with sort_every > 0;
 * steps_per_trial in [4, 100000].  Drops any captured graph.  out may be NULL. */
int pic_batch_autotune(pic_batch* b, int64_t steps_per_trial, pic_tuning* out);

/* Complete every discharge's pending step with one launch, synchronise, and report the
 * first device error of any discharge. */
int pic_batch_sync(pic_batch* b);

/* Borrow the handle of discharge k (0 <= k < n) for the per-discharge calls (moments,
 * counters, particles, fields, and pic_step to advance that discharge alone); valid until
 * pic_batch_free, which frees it.  Do not call pic_free on it. */
int pic_batch_handle(pic_batch* b, int k, pic_handle** h);

/* Number of workgroups of discharge k in batched launches (for measurement). */
int pic_batch_blocks(const pic_batch* b, int k, int* blocks);

/* Mean duration (ms) of the batched particle-pass launch over the window started by
 * pic_batch_timing(b, 1) and read by pic_batch_timing(b, 0) (HIP events on the stream). */
int pic_batch_timing(pic_batch* b, int start, double* mean_ms, int64_t* n_launches);

void pic_batch_free(pic_batch* b);

/* Message for the last error of a batch (or of its creation when b is NULL). */
const char* pic_batch_last_error(const pic_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* PIC1D_H */
