// Data layout shared by the host library (pic_api.cpp) and the gfx950 kernels
// (pic_kernels.hip).  Particle state is FP32 structure-of-arrays in HBM; the grid
// quantities that feed the Poisson solve and the electrode bookkeeping are FP64.
// Positions are stored in cell units t = x/dx in [0, n_cells]: the cloud-in-cell cell
// and weight are then exact (j = floor(t), w = t - j) and the far electrode is exactly
// t = n_cells; the resolution in metres equals that of an FP32 position in metres.
#pragma once
#include <cstdint>

namespace pic {

constexpr int kMaxProc = 16;
constexpr int kMaxProcPerSpecies = 8;
constexpr int kMaxCells = 4096;
constexpr int kBirthSortCap = 2048;   // births per step ranked by a sort in LDS; more are binned
constexpr int kNoAllocMaxPoints = 1024;   // profile points of pic_load_profiles_noalloc
constexpr int kMaxSortBlocks = 4096;  // workgroups of the periodic reordering
// Per-workgroup counters of the particle pass go to kRepSets sets (workgroup b to set
// b % kRepSets), each on its own 256-byte stretch, so that their atomics do not all
// serialise on the control block's few cache lines; the last workgroup sums the sets.
constexpr int kRepSets = 16;
constexpr int kRepStride = 32;        // 64-bit words per set
// Set 0 also holds the two species' block counters of the particle pass (kRepBlock + s); the
// last workgroup clears every set, so each launch starts them at zero.
enum : int { kRepAbs = 0, kRepColl = 4, kRepViol = 20, kRepErr = 22, kRepTicks = 23, kRepParts = 25,
             kRepDone = 27, kRepBlock = 28 };
// LDS of the particle pass's work distribution: a ring of kPassRing tagged block ids and the
// workgroup's sub-block counter (padded to 8 bytes).
constexpr int kPassRing = 8;
constexpr int kPassRingBytes = kPassRing * 8 + 8;
// The dynamic distribution's blocks go to a species' workgroups only where each holds at least
// this many of its slots (8 blocks of 4096); the host picks the dynamic pass for a single
// discharge whose workgroups start with twice that.
constexpr int64_t kPassDynMinShare = 8 * 4096;
// Charge deposit in fixed point: a particle's two cloud-in-cell weights are integers
// summing to 2^24, accumulated with integer atomics, so the node charges are exact and
// independent of the order of accumulation (bitwise reproducible runs).
constexpr float kQScale = 16777216.0f;
constexpr double kQScaleInv = 1.0 / 16777216.0;
constexpr unsigned long long kQOne = 16777216ull;
// The density moment of a sampled step is the deposit of the positions it samples (the
// charge deposit of the launch that moved the particles there, kept per species).  The second moment quantity is
// summed in LDS in integer fixed point (LDS integer atomics are far faster than
// floating-point ones), in units of 1/mscale: electron energy 2^-16 eV, ion v_x 2^-8 m/s.
// Each workgroup converts its sums to FP64 when it adds them to the window sums.
constexpr double kMomScaleE = 65536.0;
constexpr double kMomScaleI = 256.0;
// Null-collision pre-test for electrons: bins uniform in g^2 up to the end of the tables,
// each with an upper bound of the summed collision frequency over the bin.
constexpr int kNullBins = 256;

// particle-pass modes (bit set)
constexpr int kComplete = 1;   // finish the previous step: second half kick, MCC, births, moments
constexpr int kAdvance = 2;    // start the next step: first half kick, drift, absorb, deposit, solve
constexpr int kDeposit = 4;    // deposit only and solve at the current time (load / set_particles)
constexpr int kRecord = 8;     // with kComplete: write the per-slot collision decision record

// device error bits
constexpr uint32_t kErrCapacity = 1u;   // particle storage exhausted by births
constexpr uint32_t kErrNumeric = 2u;    // non-finite coordinate
constexpr uint32_t kErrBirths = 4u;     // per-step birth buffer exhausted
constexpr uint32_t kErrIds = 8u;        // 32-bit id space exhausted
constexpr uint32_t kErrSchedule = 16u;  // a wait of the work distribution reached its bound (internal)

// Control block: one per discharge, device resident, read by every kernel at launch and
// updated by the last workgroup of each launch (so it stays valid under graph replay).
struct Ctrl {
    int64_t step;                 // state time index n
    int64_t n_slots[2];           // storage in use (alive + absorbed holes)
    int64_t n_alive[2];
    int64_t next_id[2];
    int64_t particle_steps;
    unsigned long long absorbed_step[2][2];
    unsigned long long absorbed_total[2][2];
    unsigned long long absorbed_window[2][2];
    unsigned long long coll[kMaxProc];
    unsigned long long viol[2];
    unsigned long long births_total;
    unsigned long long births_lost;
    unsigned int n_births;        // births of the running launch
    unsigned int done;            // workgroups finished in the running launch
    unsigned int err;
    unsigned int cur;             // live particle buffer set (0/1); the sort flips it
    double E0_prev;
    double J_last;
    double sigma0, sigmad;
    int64_t n_samples;
    int64_t n_steps_window;
    int64_t n_periods;
    double J_period_max;
    double J_max_sum;
    int32_t period_valid;
    int32_t pad;
    unsigned long long sort_alive[2];  // alive count found by the sort histogram
    unsigned long long cost_ticks[2];  // workgroup time spent per species in the running launch
    unsigned long long cost_parts[2];  // and the slots it covered
    double cost_ratio;                 // smoothed time per electron slot / time per ion slot
    double V0;                         // RF amplitude in use [V]
};

struct ProcDev {
    int32_t kind;
    int32_t idx;        // index in the configuration (collision counters, decision codes)
    int32_t n;          // table points
    int32_t off;        // offset into the table array
    float thr;          // threshold [eV]
    float inv_de;       // 1/de [1/eV]
    float emin;         // energy floor [eV]
    float efac;         // frame energy per g^2 [eV s^2/m^2]
};

struct Params {
    // particle storage [buffer set][species]
    float* x[2][2];      // position in cell units; <= 0 marks an absorbed slot
    float* vx[2][2];
    float* vy[2][2];
    float* vz[2][2];
    uint32_t* id[2][2];
    int64_t cap[2];
    Ctrl* ctrl;
    float* E;            // node field, FP32 copy for the gather [nn]
    unsigned long long* Qs;  // node deposit per species, fixed point: 2^24 per particle [2][nn]
    unsigned long long* rep; // per-workgroup counter sets [kRepSets][kRepStride]
    double* Q_last;      // charge of the last solve [C/m^2] [nn]
    double* phi;         // node potential [V] [nn]
    double* mom;         // moment window sums [5][nn]: dens_e, dens_i, energy_e, flux_i, phi
    double mscale[2];    // fixed-point scale of the second moment quantity per species
    uint32_t* birth_parent;   // [max_births]
    unsigned long long* birth_order;   // ranking scratch: (parent id << 32 | birth index) [max_births]
    unsigned* sort_cnt;       // reordering histograms [2 n_cells + kMaxSortBlocks]
    unsigned* sort_cursor;    // their exclusive prefix sums [2 n_cells + kMaxSortBlocks]
    int8_t* dec[2];      // decision record per slot, or null
    const float* tab;    // n_gas * sigma tables [1/m]
    const float* nullbound;   // [kNullBins + 1] electron collision-frequency bounds [1/s]
    float inv_gbin;           // bins per unit g^2 [s^2/m^2]
    float pad1;
    ProcDev proc[2][kMaxProcPerSpecies];      // processes of each species, in config order
    int32_t sp_n[2];                          // processes per species
    int32_t nproc;
    int32_t n_cells;
    int32_t max_births;
    int32_t moments_every;
    int32_t steps_per_period;
    int32_t pad0;
    int32_t sort_cells[2];    // periodic reordering per species: 1 cell sort, 0 compaction only
    float ncf;           // n_cells as float: the grounded electrode in cell units
    float dt_over_dx;    // drift factor for positions in cell units
    float dt;
    float kick[2];       // 1/2 (q/m) dt
    float half_m_over_e[2];   // 1/2 m / e0 (lab energy per g^2)
    float two_e_over_m_e;     // 2 e0 / m_e
    float e_over_m_e;         // e0 / m_e
    float vT;                 // sqrt(k_B T_gas / M)
    float numax[2];
    uint32_t T[2];
    float fa[2], fb[2];       // m/(m+M), M/(m+M)
    uint32_t key0, key1;
    double dx_d;
    double eps0;
    double e0W;               // e0 * W: node charge per unit of deposited weight
    double V0, omega, dt_d;   // V0: the configured amplitude (the one in use is Ctrl::V0)
    double J0_target;         // > 0: current-driven, V0 adapted once per RF period
    unsigned long long* flux_trace;   // electrons, ions absorbed at z = 0 per step of the RF period [spp][2]
};

// Diagnostic window (samples of the completed state, off the particle pass).  node holds
// [8][nn] sums: electron weight, energy U [eV], e0 U v_x, expected ionisation rate, fast
// electrons, v_x, heating -e0 E (sum v_x), and the field.
struct DiagDev {
    double* node;
    double* fx_sample;           // [nn] this sample's v_x sums, moved into the window by the node pass
    unsigned long long* hist;    // [n_bins] electron energy histogram over [0, u_max)
    unsigned long long* counts;  // [2] electrons sampled, samples
    float bins_per_eV;
    int n_bins;
    int n_iz;                    // electron ionisation processes (P.proc[0] indices in iz)
    int iz[kMaxProcPerSpecies];
    double e0;
};

}  // namespace pic
