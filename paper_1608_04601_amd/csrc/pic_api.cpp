// Host side of the C ABI declared in include/pic1d.h: configuration checks, derived
// constants, device storage, launch sequencing, deferred error reporting and the test
// hooks.  All device work goes through the gfx950 kernels of pic_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "pic1d.h"
#include "pic_types.hpp"

namespace pic {
hipError_t launch_pass(int mode, const Params& P, int blocks, int threads, size_t lds, hipStream_t st, bool dyn);
hipError_t launch_load(const Params& P, int s, int64_t n, double vth, hipStream_t st);
hipError_t launch_sort(const Params& P, unsigned* cnt, unsigned* cursor, int blocks, int threads, hipStream_t st);
hipError_t launch_load_profile(const Params& P, int s, int64_t n, unsigned b, const double* tab, int np, double h_m,
                               hipStream_t st);
size_t diag_lds_bytes(int nn, int n_bins);
hipError_t set_diag_lds_limit(size_t bytes);
hipError_t launch_diag(const Params& P, const DiagDev& D, int blocks, hipStream_t st);
hipError_t launch_reset_window(const Params& P, hipStream_t st);
hipError_t set_pass_lds_limit(size_t bytes);
hipError_t pass_occupancy(int threads, size_t lds, int* blocks_per_cu);
hipError_t launch_pass_batch(int mode, const Params* batch, const int* seg, int nd, int blocks, int threads,
                             size_t lds, hipStream_t st);
hipError_t set_pass_batch_lds_limit(size_t bytes);
hipError_t pass_batch_occupancy(int threads, size_t lds, int* blocks_per_cu);
hipError_t launch_sort_batch(const Params* batch, const int* sseg, int nd, int blocks, int max_cells,
                             hipStream_t st);
hipError_t noalloc_scratch(int device, double** ptr, size_t* count);
}  // namespace pic

namespace {

// CODATA 2018
constexpr double kE0 = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKB = 1.380649e-23;
constexpr double kMe = 9.1093837015e-31;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_init_error;

int species_of_kind(int kind) { return kind <= PIC_E_IONIZATION ? PIC_ELECTRON : PIC_ION; }

}  // namespace

struct pic_handle {
    pic_config cfg{};
    std::vector<pic_xsec> xs;
    std::vector<std::vector<double>> tables;
    // derived (Sec. 2.1 gas density, Sec. 2.5 constant weight)
    double dx = 0, n_gas = 0, W = 0, M = 0, vT = 0;
    double mass[2] = {0, 0};
    double numax[2] = {0, 0}, pnull[2] = {0, 0};
    uint32_t T[2] = {0, 0};
    int spp = 1;
    // device
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    pic::Params P{};
    unsigned* sort_cnt = nullptr;
    unsigned* sort_cursor = nullptr;
    int8_t* dec_store[2] = {nullptr, nullptr};
    // diagnostic window (pic_diag_*), allocated by pic_diag_config
    pic::DiagDev diag{};
    int diag_capacity_bins = 0;
    double diag_umax = 0.0;
    int blocks = 1, threads = 256;
    bool dyn_pass = false;   // the pass with the dynamic work distribution (pass_dyn_kernel)
    size_t lds = 0;
    int sort_blocks = 1, sort_threads = 256;
    // sequencing
    bool pending = false;
    int since_sort = 0;
    // errors
    int status = PIC_OK;
    std::string err;
    // timing of the particle pass
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int64_t n_timed = 0;
    // captured graph of graph_steps steps (pic_set_graph), valid from reorder phase gsig and
    // pending state gpend; it leaves the phase at gend
    int64_t graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap = nullptr;   // private stream the graph is captured on
    int gsig = 0, gend = 0;
    bool gpend = false;
    int64_t graph_launches = 0;
};

namespace {

int fail(pic_handle* h, int code, const std::string& msg) {
    if (h) {
        if (h->status == PIC_OK) {
            h->status = code;
            h->err = msg;
        }
        return h->status;
    }
    g_init_error = msg;
    return code;
}

bool hip_ok(pic_handle* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    fail(h, PIC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

// Dynamic LDS of the particle pass for nn nodes and nt threads: the larger of the
// streaming layout (counters, fixed-point deposit, fixed-point moment sum, field,
// null-collision bounds, candidate queues of 128 seven-word entries per wave) and the
// epilogue layout (control block copy, three FP64 node arrays, scratch, then the
// potential or, before the solve, the birth keys and parents).
size_t pass_lds_bytes(int nn, int nt) {
    const size_t pass_lds = 32 * 4 + pic::kPassRingBytes + (size_t)nn * (8 + 8 + 4) + (size_t)(pic::kNullBins + 1) * 4 +
                            (size_t)(nt / 64) * 128 * 7 * 4;
    const size_t epi_lds = 512 + (size_t)24 * nn + 512 + std::max((size_t)8 * nn, (size_t)pic::kBirthSortCap * 8);
    return std::max(pass_lds, epi_lds);
}

// sigma_j at frame energy eps (FP64): zero below threshold, floor emin, clamp at the
// last point, linear interpolation in between.
double sigma_at(const pic_xsec& p, const std::vector<double>& tab, double eps) {
    if (eps < p.threshold_eV) return 0.0;
    const double t = std::max(eps, p.emin_eV) / p.de_eV;
    const double k = std::floor(t);
    const int n = p.n_points;
    if (k >= n - 1) return tab[n - 1];
    const int kk = (int)k;
    return tab[kk] + (tab[kk + 1] - tab[kk]) * (t - kk);
}

// Supremum over the table range of n_gas * sum_j sigma_j * g for species s.  As a function
// of the lab energy the summed cross section is piecewise linear between the union of
// all table points, thresholds and floors; on each piece (a + b eps) sqrt(eps) peaks at an
// end or at eps = -a / (3 b).
double compute_numax(const pic_handle* h, int s) {
    std::vector<int> procs;
    for (size_t j = 0; j < h->xs.size(); ++j)
        if (species_of_kind(h->xs[j].kind) == s) procs.push_back((int)j);
    if (procs.empty()) return 0.0;
    const double m = h->mass[s], M = h->M;
    std::vector<double> c(h->xs.size(), 1.0);
    double top = 0.0;
    for (int j : procs) {
        c[j] = h->xs[j].frame == PIC_FRAME_LAB ? 1.0 : M / (m + M);
        top = std::max(top, (h->xs[j].n_points - 1) * h->xs[j].de_eV / c[j]);
    }
    std::vector<double> bp = {0.0, top};
    for (int j : procs) {
        const pic_xsec& p = h->xs[j];
        for (int k = 0; k < p.n_points; ++k) bp.push_back(k * p.de_eV / c[j]);
        bp.push_back(p.threshold_eV / c[j]);
        bp.push_back(p.emin_eV / c[j]);
    }
    std::sort(bp.begin(), bp.end());
    bp.erase(std::unique(bp.begin(), bp.end()), bp.end());
    auto total_sigma = [&](double e) {
        double acc = 0.0;
        for (int j : procs) acc += sigma_at(h->xs[j], h->tables[j], c[j] * e);
        return acc;
    };
    double best = 0.0;
    auto consider = [&](double a, double b, double e) {
        const double sg = std::max(a + b * e, 0.0);
        best = std::max(best, sg * std::sqrt(2.0 * kE0 * e / m));
    };
    for (size_t k = 0; k + 1 < bp.size(); ++k) {
        const double lo = bp[k], hi = bp[k + 1];
        if (lo < 0.0 || hi > top || !(hi > lo)) continue;
        const double m1 = lo + (hi - lo) / 3.0, m2 = lo + 2.0 * (hi - lo) / 3.0;
        const double s1 = total_sigma(m1), s2 = total_sigma(m2);
        const double b = (s2 - s1) / (m2 - m1);
        const double a = s1 - b * m1;
        consider(a, b, lo);
        consider(a, b, hi);
        if (b < 0.0) {
            const double st = -a / (3.0 * b);
            if (st > lo && st < hi) consider(a, b, st);
        }
    }
    return h->n_gas * best;
}

// Electron null-collision pre-test (Sec. 2.5): for bins uniform in g^2 up to the end of
// the longest electron table, an upper bound of n_gas sum_j sigma_j g as the kernel
// evaluates it from the FP32 tables.  On a bin, each process's interpolated cross section
// is at most the largest table value between the points that bracket the bin's energies
// (both ends widened by 0.1 %), and g at most the root of the widened upper end; the sum
// is raised by another 0.1 %, which covers the FP32 rounding of the kernel's evaluation.
// A candidate with R nu_max at or above its bin's bound therefore selects no process.
// Entries beyond the last bin, and for a species without electron processes, are +inf.
std::vector<float> null_bounds(const pic_handle* h, const std::vector<float>& htab, const pic::Params& P,
                               float* inv_gbin) {
    const int nb = pic::kNullBins;
    std::vector<float> U(nb + 1, std::numeric_limits<float>::infinity());
    *inv_gbin = 0.0f;
    const int ne = P.sp_n[0];
    if (ne == 0) return U;
    double g2_top = 0.0;
    for (int k = 0; k < ne; ++k) {
        const pic::ProcDev& d = P.proc[0][k];
        const double de = 1.0 / (double)d.inv_de;
        g2_top = std::max(g2_top, (d.n - 1) * de / (double)d.efac);
    }
    if (!(g2_top > 0.0) || !std::isfinite(g2_top)) return U;
    const double width = g2_top / nb;
    *inv_gbin = (float)(1.0 / width);
    for (int b = 0; b < nb; ++b) {
        const double lo = b * width * (1.0 - 1e-3), hi = (b + 1) * width * (1.0 + 1e-3);
        double sum = 0.0;
        for (int k = 0; k < ne; ++k) {
            const pic::ProcDev& d = P.proc[0][k];
            const double tlo = std::max((double)d.efac * lo, (double)d.emin) * (double)d.inv_de;
            const double thi = std::max((double)d.efac * hi, (double)d.emin) * (double)d.inv_de;
            const int k0 = std::min(std::max((int)std::floor(tlo), 0), d.n - 1);
            const int k1 = std::min((int)std::ceil(thi) + 1, d.n - 1);
            double mx = 0.0;
            for (int q = k0; q <= k1; ++q) mx = std::max(mx, (double)htab[(size_t)d.off + q]);
            sum += mx;
        }
        const double bound = sum * std::sqrt(hi) * (1.0 + 1e-3);
        float f = (float)bound;
        if ((double)f < bound) f = std::nextafter(f, std::numeric_limits<float>::infinity());
        U[b] = f;
    }
    return U;
}

std::string validate(const pic_config* c) {
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    auto nonneg = [](double v) { return std::isfinite(v) && v >= 0.0; };
    if (!c) return "config is NULL";
    if (!pos(c->gap_m)) return "gap_m must be > 0";
    if (!pos(c->pressure_Pa)) return "pressure_Pa must be > 0";
    if (!pos(c->gas_temperature_K)) return "gas_temperature_K must be > 0";
    if (!pos(c->gas_mass_amu)) return "gas_mass_amu must be > 0";
    if (!std::isfinite(c->rf_voltage_V)) return "rf_voltage_V must be finite";
    if (!pos(c->rf_frequency_Hz)) return "rf_frequency_Hz must be > 0";
    if (!pos(c->dt_s)) return "dt_s must be > 0";
    if (!nonneg(c->n_init_m3)) return "n_init_m3 must be >= 0";
    if (!nonneg(c->te_init_eV) || !nonneg(c->ti_init_eV)) return "initial temperatures must be >= 0";
    if (c->n_cells < 2 || c->n_cells > PIC_MAX_CELLS) return "n_cells must be in [2, 4096]";
    if (c->n_xsec < 0 || c->n_xsec > PIC_MAX_PROCESSES) return "n_xsec must be in [0, 16]";
    if (c->n_xsec > 0 && !c->xsec) return "xsec is NULL";
    for (int s = 0; s < 2; ++s) {
        if (c->capacity[s] < 1 || c->capacity[s] >= (int64_t(1) << 31)) return "capacity must be in [1, 2^31)";
        if (c->n_init_super[s] < 0 || c->n_init_super[s] > c->capacity[s])
            return "n_init_super must be in [0, capacity]";
    }
    if (c->n_init_super[0] < 1) return "n_init_super[0] must be > 0 (it sets the weight)";
    if (c->sort_every < 0) return "sort_every must be >= 0";
    if (c->moments_every < 1) return "moments_every must be >= 1";
    if (c->max_births_per_step < 1) return "max_births_per_step must be >= 1";
    if (c->launch_blocks < 0 || c->launch_blocks > 65536) return "launch_blocks must be in [0, 65536]";
    if (c->electron_order < -1 || c->electron_order > 1) return "electron_order must be -1, 0 or 1";
    if (c->reserved != 0) return "reserved must be 0";
    if (!std::isfinite(c->j0_target_A_m2) || c->j0_target_A_m2 < 0.0) return "j0_target_A_m2 must be finite and >= 0";
    int per_species[2] = {0, 0};
    for (int j = 0; j < c->n_xsec; ++j) {
        const pic_xsec& p = c->xsec[j];
        if (p.kind >= PIC_E_ELASTIC && p.kind <= PIC_I_BACKWARD &&
            ++per_species[species_of_kind(p.kind)] > pic::kMaxProcPerSpecies)
            return "at most 8 processes per species";
        if (p.kind < PIC_E_ELASTIC || p.kind > PIC_I_BACKWARD) return "xsec kind out of range";
        if (p.frame != PIC_FRAME_LAB && p.frame != PIC_FRAME_CM) return "xsec frame out of range";
        if (p.n_points < 2 || p.n_points > (1 << 22)) return "xsec n_points must be in [2, 2^22]";
        if (p.reserved != 0) return "xsec reserved must be 0";
        if (!nonneg(p.threshold_eV) || !pos(p.de_eV) || !nonneg(p.emin_eV)) return "xsec energies invalid";
        if (!p.sigma_m2) return "xsec sigma_m2 is NULL";
        for (int k = 0; k < p.n_points; ++k)
            if (!nonneg(p.sigma_m2[k])) return "xsec sigma_m2 must be finite and >= 0";
    }
    return "";
}

template <typename T>
bool dev_alloc(pic_handle* h, T** out, size_t count) {
    *out = nullptr;
    if (count == 0) return true;
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        fail(h, PIC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        return false;
    }
    h->allocs.push_back(p);
    *out = static_cast<T*>(p);
    return true;
}

void drop_graph(pic_handle* h) {
    if (h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
}

void release(pic_handle* h) {
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->cap) {
        (void)hipStreamDestroy(h->cap);
        h->cap = nullptr;
    }
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    h->ev.clear();
}

int check_device(pic_handle* h) {
    if (h->status) return h->status;
    if (!hip_ok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize")) return h->status;
    unsigned err = 0;
    if (!hip_ok(h, hipMemcpy(&err, &h->P.ctrl->err, sizeof(err), hipMemcpyDeviceToHost), "hipMemcpy(err)"))
        return h->status;
    if (err & (pic::kErrCapacity | pic::kErrBirths | pic::kErrIds)) {
        std::string what = (err & pic::kErrCapacity) ? "particle storage exhausted"
                           : (err & pic::kErrBirths) ? "per-step birth buffer exhausted"
                                                     : "32-bit particle id space exhausted";
        return fail(h, PIC_ECAPACITY, what);
    }
    if (err & pic::kErrNumeric) return fail(h, PIC_ENUMERIC, "non-finite particle coordinate");
    if (err & pic::kErrSchedule) return fail(h, PIC_EHIP, "particle pass: work distribution wait exceeded its bound");
    return PIC_OK;
}

int launch_pass_timed(pic_handle* h, int mode) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool t = h->timing && (mode & pic::kAdvance);
    if (t) {
        const size_t k = (size_t)h->n_timed * 2;
        if (k + 2 > h->ev.size()) {
            if (h->ev.size() >= 2 * 8192) {
                h->timing = false;
            } else {
                for (int q = 0; q < 2; ++q) {
                    hipEvent_t e;
                    if (!hip_ok(h, hipEventCreate(&e), "hipEventCreate")) return h->status;
                    h->ev.push_back(e);
                }
            }
        }
        if (h->timing) {
            a = h->ev[k];
            b = h->ev[k + 1];
            if (!hip_ok(h, hipEventRecord(a, h->stream), "hipEventRecord")) return h->status;
        }
    }
    const int launch_mode = mode | ((h->P.dec[0] && (mode & pic::kComplete)) ? pic::kRecord : 0);
    if (!hip_ok(h, pic::launch_pass(launch_mode, h->P, h->blocks, h->threads, h->lds, h->stream, h->dyn_pass),
                "pass_kernel launch"))
        return h->status;
    if (t && h->timing) {
        if (!hip_ok(h, hipEventRecord(b, h->stream), "hipEventRecord")) return h->status;
        h->n_timed += 1;
    }
    return PIC_OK;
}

int complete_pending(pic_handle* h) {
    if (!h->pending) return PIC_OK;
    const int rc = launch_pass_timed(h, pic::kComplete);
    if (rc) return rc;
    h->pending = false;
    return PIC_OK;
}

int read_ctrl(pic_handle* h, pic::Ctrl* c) {
    if (!hip_ok(h, hipMemcpyAsync(c, h->P.ctrl, sizeof(*c), hipMemcpyDeviceToHost, h->stream), "hipMemcpy(ctrl)"))
        return h->status;
    if (!hip_ok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize")) return h->status;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_init(const pic_config* cfg, void* hip_stream, pic_handle** out) {
    if (!out) {
        g_init_error = "out is NULL";
        return PIC_EINVAL;
    }
    *out = nullptr;
    const std::string bad = validate(cfg);
    if (!bad.empty()) {
        g_init_error = bad;
        return PIC_EINVAL;
    }
    pic_handle* h = new (std::nothrow) pic_handle();
    if (!h) {
        g_init_error = "out of host memory";
        return PIC_ENOMEM;
    }
    h->cfg = *cfg;
    for (int j = 0; j < cfg->n_xsec; ++j) {
        h->xs.push_back(cfg->xsec[j]);
        h->tables.emplace_back(cfg->xsec[j].sigma_m2, cfg->xsec[j].sigma_m2 + cfg->xsec[j].n_points);
        h->xs.back().sigma_m2 = nullptr;
    }
    h->cfg.xsec = nullptr;
    const pic_config& c = h->cfg;
    const int nc = c.n_cells, nn = nc + 1;

    // ---- derived constants
    h->dx = c.gap_m / nc;
    h->n_gas = c.pressure_Pa / (kKB * c.gas_temperature_K);
    h->W = c.n_init_m3 * c.gap_m / (double)c.n_init_super[0];
    h->M = c.gas_mass_amu * kAmu;
    h->mass[0] = kMe;
    h->mass[1] = h->M;
    h->vT = std::sqrt(kKB * c.gas_temperature_K / h->M);
    for (int s = 0; s < 2; ++s) {
        h->numax[s] = compute_numax(h, s);
        h->pnull[s] = -std::expm1(-h->numax[s] * c.dt_s);
        h->T[s] = (uint32_t)std::nearbyint(h->pnull[s] * 16777216.0);
    }
    h->spp = std::max(1L, std::lround(1.0 / (c.rf_frequency_Hz * c.dt_s)));

    // ---- stream
    if (!hip_ok(h, hipGetDevice(&h->device), "hipGetDevice")) goto fail_init;
    {   // the no-allocation loader's staging: its address on this device, looked up once
        double* sp = nullptr;
        size_t sn = 0;
        if (!hip_ok(h, pic::noalloc_scratch(h->device, &sp, &sn), "scratch address")) goto fail_init;
    }
    h->stream = static_cast<hipStream_t>(hip_stream);   // NULL: the device's null stream

    {
        pic::Params& P = h->P;
        const int nbuf = c.sort_every > 0 ? 2 : 1;
        for (int b = 0; b < nbuf; ++b)
            for (int s = 0; s < 2; ++s) {
                const size_t cap = (size_t)c.capacity[s];
                if (!dev_alloc(h, &P.x[b][s], cap) || !dev_alloc(h, &P.vx[b][s], cap) ||
                    !dev_alloc(h, &P.vy[b][s], cap) || !dev_alloc(h, &P.vz[b][s], cap) ||
                    !dev_alloc(h, &P.id[b][s], cap))
                    goto fail_init;
            }
        for (int s = 0; s < 2; ++s) P.cap[s] = c.capacity[s];
        size_t ntab = 0;
        for (const pic_xsec& p : h->xs) ntab += (size_t)p.n_points;
        float* tab = nullptr;
        float* nullbound = nullptr;
        if (!dev_alloc(h, &P.ctrl, 1) || !dev_alloc(h, &P.rep, (size_t)pic::kRepSets * pic::kRepStride) ||
            !dev_alloc(h, &P.E, nn) || !dev_alloc(h, &P.Qs, (size_t)2 * nn) ||
            !dev_alloc(h, &nullbound, (size_t)pic::kNullBins + 1) ||
            !dev_alloc(h, &P.Q_last, nn) || !dev_alloc(h, &P.phi, nn) || !dev_alloc(h, &P.mom, (size_t)5 * nn) ||
            !dev_alloc(h, &P.birth_parent, (size_t)c.max_births_per_step) ||
            !dev_alloc(h, &P.birth_order, (size_t)c.max_births_per_step) || !dev_alloc(h, &tab, std::max<size_t>(ntab, 1)) ||
            !dev_alloc(h, &h->sort_cnt, (size_t)2 * nc + pic::kMaxSortBlocks) ||
            !dev_alloc(h, &h->sort_cursor, (size_t)2 * nc + pic::kMaxSortBlocks) ||
            !dev_alloc(h, &P.flux_trace, (size_t)2 * h->spp))
            goto fail_init;
        P.sort_cnt = h->sort_cnt;
        P.sort_cursor = h->sort_cursor;
        P.tab = tab;
        P.nullbound = nullbound;
        std::vector<float> htab;
        htab.reserve(ntab);
        P.nproc = (int)h->xs.size();
        for (size_t j = 0; j < h->xs.size(); ++j) {
            const pic_xsec& p = h->xs[j];
            const int s = species_of_kind(p.kind);
            pic::ProcDev& d = P.proc[s][P.sp_n[s]++];
            const double m = h->mass[s];
            const double m_frame = p.frame == PIC_FRAME_LAB ? m : m * h->M / (m + h->M);
            d.kind = p.kind;
            d.idx = (int)j;
            d.n = p.n_points;
            d.off = (int)htab.size();
            d.thr = (float)p.threshold_eV;
            d.inv_de = (float)(1.0 / p.de_eV);
            d.emin = (float)p.emin_eV;
            d.efac = (float)(0.5 * m_frame / kE0);
            for (double v : h->tables[j]) htab.push_back((float)(h->n_gas * v));
        }
        const std::vector<float> hbound = null_bounds(h, htab, P, &P.inv_gbin);
        P.n_cells = nc;
        P.max_births = c.max_births_per_step;
        P.moments_every = c.moments_every;
        P.steps_per_period = h->spp;
        P.ncf = (float)nc;
        P.dt_over_dx = (float)(c.dt_s / h->dx);
        P.dt = (float)c.dt_s;
        const double q[2] = {-kE0, kE0};
        for (int s = 0; s < 2; ++s) {
            P.kick[s] = (float)(0.5 * q[s] / h->mass[s] * c.dt_s);
            P.half_m_over_e[s] = (float)(0.5 * h->mass[s] / kE0);
            P.numax[s] = (float)h->numax[s];
            P.T[s] = h->T[s];
            P.fa[s] = (float)(h->mass[s] / (h->mass[s] + h->M));
            P.fb[s] = (float)(h->M / (h->mass[s] + h->M));
        }
        P.two_e_over_m_e = (float)(2.0 * kE0 / kMe);
        P.e_over_m_e = (float)(kE0 / kMe);
        P.vT = (float)h->vT;
        P.key0 = (uint32_t)(c.seed & 0xFFFFFFFFu);
        P.key1 = (uint32_t)(c.seed >> 32);
        P.dx_d = h->dx;
        P.eps0 = kEps0;
        P.e0W = kE0 * h->W;
        P.V0 = c.rf_voltage_V;
        P.J0_target = c.j0_target_A_m2;
        P.omega = 2.0 * kPi * c.rf_frequency_Hz;
        P.dt_d = c.dt_s;
        // periodic reordering: ions by cell; electrons by cell only while they stay near
        // their cell over a sort interval (else cell order is lost within a few steps and
        // the sort's scattered writes cost more than it saves)
        {
            const double v3 = std::sqrt(3.0 * kE0 / kMe);
            const double cells = (double)std::max(c.sort_every, 1) * c.dt_s * v3 / h->dx;
            P.sort_cells[0] = c.electron_order == 1 || (c.electron_order == -1 && cells <= 16.0);
            P.sort_cells[1] = 1;
        }
        P.mscale[0] = pic::kMomScaleE;
        P.mscale[1] = pic::kMomScaleI;

        // launch shape: one workgroup per contiguous particle range; LDS holds the node
        // field, the private deposit and moment grids, the null-collision bounds and the
        // candidate queue
        h->threads = nn <= 1025 ? 256 : 1024;
        h->lds = pass_lds_bytes(nn, h->threads);
        const int64_t total = c.n_init_super[0] + c.n_init_super[1];
        h->sort_threads = 1024;
        h->sort_blocks = (int)std::min<int64_t>(pic::kMaxSortBlocks, std::max<int64_t>(2, (total + 8191) / 8192));
        if (!hip_ok(h, pic::set_pass_lds_limit(h->lds), "hipFuncSetAttribute")) goto fail_init;
        if (c.launch_blocks > 0) {
            h->blocks = c.launch_blocks;
        } else {
            // Workgroups resident at once (LDS and registers permitting) on all compute
            // units, and at least 8 particles per thread.  The device splits them between
            // the species by measured cost, so one round is enough.
            int cus = 0, per_cu = 0;
            if (!hip_ok(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device),
                        "hipDeviceGetAttribute") ||
                !hip_ok(h, pic::pass_occupancy(h->threads, h->lds, &per_cu), "occupancy"))
                goto fail_init;
            const int64_t resident = std::max<int64_t>(1, (int64_t)cus * std::max(per_cu, 1));
            const int64_t per_block = (int64_t)h->threads * 8;
            const int64_t want = std::max<int64_t>(1, (total + per_block - 1) / per_block);
            h->blocks = (int)std::min(want, resident);
        }
        // Large shares per workgroup: the dynamic work distribution keeps the workgroups
        // together (smaller ones keep the static cut, which was faster there).
        h->dyn_pass = h->blocks > 1 && total / h->blocks >= 2 * pic::kPassDynMinShare;

        if (!hip_ok(h, hipMemcpyAsync(tab, htab.data(), htab.size() * sizeof(float), hipMemcpyHostToDevice, h->stream),
                    "upload tables") ||
            !hip_ok(h, hipMemcpyAsync(nullbound, hbound.data(), hbound.size() * sizeof(float), hipMemcpyHostToDevice,
                                      h->stream),
                    "upload null-collision bounds"))
            goto fail_init;
        pic::Ctrl c0{};
        for (int s = 0; s < 2; ++s) {
            c0.n_slots[s] = c.n_init_super[s];
            c0.n_alive[s] = c.n_init_super[s];
            c0.next_id[s] = c.n_init_super[s];
        }
        c0.period_valid = 1;
        c0.cost_ratio = 1.0;
        c0.V0 = c.rf_voltage_V;
        if (!hip_ok(h, hipMemcpyAsync(P.ctrl, &c0, sizeof(c0), hipMemcpyHostToDevice, h->stream), "upload ctrl") ||
            !hip_ok(h, hipMemsetAsync(P.Qs, 0, 2 * nn * sizeof(unsigned long long), h->stream), "zero Q") ||
            !hip_ok(h, hipMemsetAsync(P.rep, 0, pic::kRepSets * pic::kRepStride * sizeof(unsigned long long), h->stream),
                    "zero counter sets") ||
            !hip_ok(h, hipMemsetAsync(P.mom, 0, 5 * nn * sizeof(double), h->stream), "zero moments") ||
            !hip_ok(h, hipMemsetAsync(P.flux_trace, 0, sizeof(unsigned long long) * 2 * (size_t)h->spp, h->stream),
                    "zero flux trace") ||
            !hip_ok(h, hipMemsetAsync(h->sort_cnt, 0, (2 * nc + pic::kMaxSortBlocks) * sizeof(unsigned), h->stream),
                    "zero sort counts"))
            goto fail_init;
        const double temps[2] = {c.te_init_eV, c.ti_init_eV};
        for (int s = 0; s < 2; ++s) {
            const double vth = std::sqrt(kE0 * temps[s] / h->mass[s]);
            if (!hip_ok(h, pic::launch_load(P, s, c.n_init_super[s], vth, h->stream), "load_kernel"))
                goto fail_init;
        }
        if (launch_pass_timed(h, pic::kDeposit)) goto fail_init;
        if (!hip_ok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize")) goto fail_init;
    }
    *out = h;
    return PIC_OK;

fail_init:
    g_init_error = h->err;
    {
        const int code = h->status ? h->status : PIC_EHIP;
        release(h);
        delete h;
        return code;
    }
}

namespace {
// One step: the particle pass (completing the previous step if it is pending), then the
// periodic reordering when due.
int solo_one_step(pic_handle* h) {
    const int mode = pic::kAdvance | (h->pending ? pic::kComplete : 0);
    if (launch_pass_timed(h, mode)) return h->status;
    h->pending = true;
    if (h->cfg.sort_every > 0 && ++h->since_sort >= h->cfg.sort_every) {
        if (!hip_ok(h, pic::launch_sort(h->P, h->sort_cnt, h->sort_cursor, h->sort_blocks, h->sort_threads, h->stream),
                    "sort launch"))
            return h->status;
        h->since_sort = 0;
    }
    return PIC_OK;
}

// Records graph_steps steps from the current reorder phase and pending state into a graph,
// on a private stream.  Nothing runs; the host-side phase and pending flag are put back.
int solo_capture(pic_handle* h) {
    drop_graph(h);
    if (!h->cap && !hip_ok(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "hipStreamCreateWithFlags"))
        return h->status;
    const int sig = h->since_sort;
    const bool pend = h->pending;
    const hipStream_t user = h->stream;
    h->stream = h->cap;
    hipGraph_t g = nullptr;
    int rc = PIC_OK;
    if (!hip_ok(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture")) {
        rc = h->status;
    } else {
        for (int64_t k = 0; k < h->graph_steps && rc == PIC_OK; ++k) rc = solo_one_step(h);
        const hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (rc == PIC_OK && !hip_ok(h, e, "hipStreamEndCapture")) rc = h->status;
    }
    h->gend = h->since_sort;
    h->since_sort = sig;
    h->pending = pend;
    h->stream = user;
    if (rc == PIC_OK && !hip_ok(h, hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0), "hipGraphInstantiate")) {
        h->gexec = nullptr;
        rc = h->status;
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc == PIC_OK) {
        h->gsig = sig;
        h->gpend = pend;
    }
    return rc;
}
}  // namespace

int pic_step(pic_handle* h, int64_t n_steps) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (n_steps < 0) return fail(h, PIC_EINVAL, "n_steps must be >= 0");
    int64_t k = 0;
    while (k < n_steps) {
        if (h->graph_steps > 0 && n_steps - k >= h->graph_steps && !h->timing) {
            if ((!h->gexec || h->pending != h->gpend || h->since_sort != h->gsig) && solo_capture(h)) return h->status;
            if (!hip_ok(h, hipGraphLaunch(h->gexec, h->stream), "hipGraphLaunch")) return h->status;
            h->since_sort = h->gend;
            h->pending = true;
            ++h->graph_launches;
            k += h->graph_steps;
            continue;
        }
        if (solo_one_step(h)) return h->status;
        ++k;
    }
    return PIC_OK;
}

int pic_set_graph(pic_handle* h, int64_t steps_per_graph) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (steps_per_graph < 0 || steps_per_graph > 100000)
        return fail(h, PIC_EINVAL, "steps_per_graph must be in [0, 100000]");
    if (!hip_ok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize")) return h->status;
    drop_graph(h);
    h->graph_steps = steps_per_graph;
    h->graph_launches = 0;
    return PIC_OK;
}

int pic_graph_launches(const pic_handle* h, int64_t* n) {
    if (!h || !n) return PIC_EINVAL;
    *n = h->graph_launches;
    return PIC_OK;
}

int pic_launch_shape(const pic_handle* h, int* blocks, int* threads, int* dynamic) {
    if (!h) return PIC_EINVAL;
    if (blocks) *blocks = h->blocks;
    if (threads) *threads = h->threads;
    if (dynamic) *dynamic = h->dyn_pass ? 1 : 0;
    return PIC_OK;
}

int pic_sync(pic_handle* h) {
    if (!h) return PIC_EINVAL;
    return check_device(h);
}

int pic_moments(pic_handle* h, pic_moments_out* out, int reset) {
    if (!h || !out) return h ? fail(h, PIC_EINVAL, "out is NULL") : PIC_EINVAL;
    if (h->status) return h->status;
    const int nn = h->cfg.n_cells + 1;
    if (out->n_nodes != nn) return fail(h, PIC_EINVAL, "n_nodes must equal n_cells + 1");
    if (complete_pending(h)) return h->status;
    if (check_device(h)) return h->status;
    pic::Ctrl c;
    if (read_ctrl(h, &c)) return h->status;
    std::vector<double> mom((size_t)5 * nn);
    if (!hip_ok(h, hipMemcpy(mom.data(), h->P.mom, mom.size() * sizeof(double), hipMemcpyDeviceToHost), "read moments"))
        return h->status;
    const double N = (double)std::max<int64_t>(c.n_samples, 1);
    for (int i = 0; i < nn; ++i) {
        const double V = (i == 0 || i == nn - 1) ? 0.5 * h->dx : h->dx;
        const double de = mom[i], di = mom[nn + i], en = mom[2 * nn + i], fl = mom[3 * nn + i], ph = mom[4 * nn + i];
        if (out->n_e_m3) out->n_e_m3[i] = h->W * de / (V * N);
        if (out->n_i_m3) out->n_i_m3[i] = h->W * di / (V * N);
        if (out->mean_energy_e_eV) out->mean_energy_e_eV[i] = de > 0.0 ? en / de : NAN;
        if (out->flux_i_m2s) out->flux_i_m2s[i] = h->W * fl / (V * N);
        if (out->phi_V) out->phi_V[i] = ph / N;
    }
    out->n_samples = c.n_samples;
    out->n_steps = c.n_steps_window;
    out->window_s = (double)c.n_steps_window * h->cfg.dt_s;
    out->J0_A_m2 = c.n_periods > 0 ? c.J_max_sum / (double)c.n_periods : NAN;
    out->flux_i_powered_m2s = out->window_s > 0 ? h->W * (double)c.absorbed_window[1][0] / out->window_s : NAN;
    for (int s = 0; s < 2; ++s)
        for (int e = 0; e < 2; ++e) out->absorbed[s][e] = (int64_t)c.absorbed_window[s][e];
    if (reset) {
        if (!hip_ok(h, pic::launch_reset_window(h->P, h->stream), "reset_window")) return h->status;
        if (check_device(h)) return h->status;
    }
    return PIC_OK;
}

void pic_free(pic_handle* h) {
    if (!h) return;
    release(h);
    delete h;
}

const char* pic_last_error(const pic_handle* h) {
    if (!h) return g_init_error.c_str();
    return h->err.c_str();
}

int pic_get_counters(pic_handle* h, pic_counters* out) {
    if (!h || !out) return h ? fail(h, PIC_EINVAL, "out is NULL") : PIC_EINVAL;
    if (h->status) return h->status;
    if (complete_pending(h)) return h->status;
    if (check_device(h)) return h->status;
    pic::Ctrl c;
    if (read_ctrl(h, &c)) return h->status;
    std::memset(out, 0, sizeof(*out));
    out->step = c.step;
    for (int s = 0; s < 2; ++s) {
        out->n_alive[s] = c.n_alive[s];
        out->n_slots[s] = c.n_slots[s];
        out->next_id[s] = c.next_id[s];
        out->numax_violations[s] = (int64_t)c.viol[s];
        for (int e = 0; e < 2; ++e) out->absorbed_total[s][e] = (int64_t)c.absorbed_total[s][e];
    }
    out->particle_steps = c.particle_steps;
    for (int j = 0; j < PIC_MAX_PROCESSES; ++j) out->collisions[j] = (int64_t)c.coll[j];
    out->births_total = (int64_t)c.births_total;
    out->J_last_A_m2 = c.J_last;
    out->sigma0_C_m2 = c.sigma0;
    out->sigmad_C_m2 = c.sigmad;
    out->V0_V = c.V0;
    return PIC_OK;
}

int pic_get_derived(const pic_handle* h, pic_derived* out) {
    if (!h || !out) return PIC_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->dx_m = h->dx;
    out->n_gas_m3 = h->n_gas;
    out->weight_m2 = h->W;
    out->ion_mass_kg = h->M;
    out->v_thermal_gas_ms = h->vT;
    for (int s = 0; s < 2; ++s) {
        out->numax_s[s] = h->numax[s];
        out->p_null[s] = h->pnull[s];
        out->threshold[s] = h->T[s];
    }
    out->steps_per_period = h->spp;
    return PIC_OK;
}

int pic_get_particles(pic_handle* h, int species, double* x, float* vx, float* vy, float* vz, uint32_t* id,
                      int64_t capacity, int64_t* n_out) {
    if (!h || !n_out) return h ? fail(h, PIC_EINVAL, "n_out is NULL") : PIC_EINVAL;
    if (h->status) return h->status;
    if (species != 0 && species != 1) return fail(h, PIC_EINVAL, "species must be 0 or 1");
    if (complete_pending(h)) return h->status;
    if (check_device(h)) return h->status;
    pic::Ctrl c;
    if (read_ctrl(h, &c)) return h->status;
    const int64_t ns = c.n_slots[species];
    const unsigned b = c.cur;
    std::vector<float> hx(ns), hvx(ns), hvy(ns), hvz(ns);
    std::vector<uint32_t> hid(ns);
    const pic::Params& P = h->P;
    if (ns > 0 &&
        (!hip_ok(h, hipMemcpy(hx.data(), P.x[b][species], ns * 4, hipMemcpyDeviceToHost), "copy x") ||
         !hip_ok(h, hipMemcpy(hvx.data(), P.vx[b][species], ns * 4, hipMemcpyDeviceToHost), "copy vx") ||
         !hip_ok(h, hipMemcpy(hvy.data(), P.vy[b][species], ns * 4, hipMemcpyDeviceToHost), "copy vy") ||
         !hip_ok(h, hipMemcpy(hvz.data(), P.vz[b][species], ns * 4, hipMemcpyDeviceToHost), "copy vz") ||
         !hip_ok(h, hipMemcpy(hid.data(), P.id[b][species], ns * 4, hipMemcpyDeviceToHost), "copy id")))
        return h->status;
    int64_t n = 0;
    for (int64_t i = 0; i < ns; ++i) n += hx[i] > 0.0f;
    *n_out = n;
    if (!x && !vx && !vy && !vz && !id) return PIC_OK;
    if (capacity < n) return fail(h, PIC_EINVAL, "capacity too small for the alive particles");
    int64_t k = 0;
    for (int64_t i = 0; i < ns; ++i) {
        if (!(hx[i] > 0.0f)) continue;
        if (x) x[k] = (double)hx[i] * h->dx;
        if (vx) vx[k] = hvx[i];
        if (vy) vy[k] = hvy[i];
        if (vz) vz[k] = hvz[i];
        if (id) id[k] = hid[i];
        ++k;
    }
    return PIC_OK;
}

int pic_set_particles(pic_handle* h, int species, const double* x, const float* vx, const float* vy, const float* vz,
                      const uint32_t* id, int64_t n, uint32_t next_id, int64_t step) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (species != 0 && species != 1) return fail(h, PIC_EINVAL, "species must be 0 or 1");
    if (n < 0 || n > h->cfg.capacity[species]) return fail(h, PIC_EINVAL, "n must be in [0, capacity]");
    if (step < 0) return fail(h, PIC_EINVAL, "step must be >= 0");
    if (n > 0 && (!x || !vx || !vy || !vz || !id)) return fail(h, PIC_EINVAL, "particle arrays are NULL");
    const float ncf = (float)h->cfg.n_cells;
    std::vector<float> t(n);
    for (int64_t i = 0; i < n; ++i) {
        if (!(x[i] > 0.0 && x[i] < h->cfg.gap_m)) return fail(h, PIC_EINVAL, "x must be in (0, d)");
        t[i] = (float)(x[i] / h->dx);
        if (!(t[i] < ncf)) t[i] = std::nextafter(ncf, 0.0f);
        if (!(t[i] > 0.0f)) t[i] = std::numeric_limits<float>::denorm_min();
        if (!std::isfinite(vx[i]) || !std::isfinite(vy[i]) || !std::isfinite(vz[i]))
            return fail(h, PIC_EINVAL, "velocities must be finite");
        if (id[i] >= next_id) return fail(h, PIC_EINVAL, "ids must be < next_id");
    }
    if (complete_pending(h)) return h->status;
    if (check_device(h)) return h->status;
    pic::Ctrl c;
    if (read_ctrl(h, &c)) return h->status;
    const unsigned b = c.cur;
    const pic::Params& P = h->P;
    if (n > 0 &&
        (!hip_ok(h, hipMemcpy(P.x[b][species], t.data(), n * 4, hipMemcpyHostToDevice), "copy x") ||
         !hip_ok(h, hipMemcpy(P.vx[b][species], vx, n * 4, hipMemcpyHostToDevice), "copy vx") ||
         !hip_ok(h, hipMemcpy(P.vy[b][species], vy, n * 4, hipMemcpyHostToDevice), "copy vy") ||
         !hip_ok(h, hipMemcpy(P.vz[b][species], vz, n * 4, hipMemcpyHostToDevice), "copy vz") ||
         !hip_ok(h, hipMemcpy(P.id[b][species], id, n * 4, hipMemcpyHostToDevice), "copy id")))
        return h->status;
    c.n_slots[species] = n;
    c.n_alive[species] = n;
    c.next_id[species] = next_id == 0 ? 0 : (int64_t)next_id;
    c.step = step;
    if (!hip_ok(h, hipMemcpy(h->P.ctrl, &c, sizeof(c), hipMemcpyHostToDevice), "write ctrl")) return h->status;
    if (!hip_ok(h, hipMemset(h->P.Qs, 0, 2 * (h->cfg.n_cells + 1) * sizeof(unsigned long long)), "zero Q"))
        return h->status;
    if (launch_pass_timed(h, pic::kDeposit)) return h->status;
    return check_device(h);
}

namespace {
// Checks the warm-start profiles and the handle's state (not stepped); reads the control
// block into *c.
int check_profiles(pic_handle* h, int32_t n_points, const double* n_e, const double* n_i,
                   const double* mean_energy_e_eV, const double* flux_i, pic::Ctrl* c) {
    if (!n_e || !n_i || !mean_energy_e_eV || !flux_i) return fail(h, PIC_EINVAL, "profile arrays are NULL");
    for (int j = 0; j < n_points; ++j) {
        if (!std::isfinite(n_e[j]) || !std::isfinite(n_i[j]) || !std::isfinite(mean_energy_e_eV[j]) ||
            !std::isfinite(flux_i[j]))
            return fail(h, PIC_EINVAL, "profiles must be finite");
        if (n_e[j] < 0.0 || n_i[j] < 0.0 || mean_energy_e_eV[j] < 0.0)
            return fail(h, PIC_EINVAL, "densities and the mean energy must be >= 0");
    }
    if (h->pending) return fail(h, PIC_ESTATE, "the discharge has already been stepped");
    if (check_device(h)) return h->status;
    if (read_ctrl(h, c)) return h->status;
    if (c->step != 0) return fail(h, PIC_ESTATE, "the discharge has already been stepped");
    return PIC_OK;
}

// Loader table of species s on host memory t[4 * n_points]: cumulative integral of the
// density (trapezoids), density, thermal speed squared per component, mean v_x.  Returns the
// particle count round(integral / W) in *count, or an error.
int profile_table(pic_handle* h, int s, int32_t n_points, const double* n_e, const double* n_i,
                  const double* mean_energy_e_eV, const double* flux_i, double* t, int64_t* count) {
    const double hm = h->cfg.gap_m / (double)(n_points - 1);
    const double M = h->cfg.gas_mass_amu * kAmu;
    const double* dens = s == 0 ? n_e : n_i;
    t[0] = 0.0;
    for (int j = 1; j < n_points; ++j) t[j] = t[j - 1] + 0.5 * (dens[j - 1] + dens[j]) * hm;
    for (int j = 0; j < n_points; ++j) {
        t[n_points + j] = dens[j];
        t[2 * n_points + j] = s == 0 ? kE0 * (2.0 / 3.0) * mean_energy_e_eV[j] / kMe
                                     : kKB * h->cfg.gas_temperature_K / M;
        t[3 * n_points + j] = (s == 1 && n_i[j] > 0.0) ? flux_i[j] / n_i[j] : 0.0;
    }
    *count = (int64_t)std::floor(t[n_points - 1] / h->W + 0.5);
    if (*count < 1) return fail(h, PIC_EINVAL, "a density profile holds less than one particle");
    if (*count > h->cfg.capacity[s]) return fail(h, PIC_ECAPACITY, "the profiles need more particles than capacity");
    return PIC_OK;
}

// Device half of the warm-start load: the tables of both species are in dtab (species s at
// 4 * n_points * s); draws the particles, sets the counts and solves the field at t = 0.
int load_from_tables(pic_handle* h, pic::Ctrl& c, int32_t n_points, const double* dtab, const int64_t count[2]) {
    const double hm = h->cfg.gap_m / (double)(n_points - 1);
    const unsigned b = c.cur;
    for (int s = 0; s < 2; ++s)
        if (!hip_ok(h, pic::launch_load_profile(h->P, s, count[s], b, dtab + (size_t)4 * n_points * s, n_points, hm,
                                                h->stream),
                    "load_profile_kernel"))
            return h->status;
    for (int s = 0; s < 2; ++s) {
        c.n_slots[s] = count[s];
        c.n_alive[s] = count[s];
        c.next_id[s] = count[s];
    }
    if (!hip_ok(h, hipMemcpyAsync(h->P.ctrl, &c, sizeof(c), hipMemcpyHostToDevice, h->stream), "write ctrl") ||
        !hip_ok(h, hipMemsetAsync(h->P.Qs, 0, 2 * (h->cfg.n_cells + 1) * sizeof(unsigned long long), h->stream),
                "zero Q") ||
        !hip_ok(h, pic::launch_pass(pic::kDeposit, h->P, h->blocks, h->threads, h->lds, h->stream, h->dyn_pass),
                "deposit pass"))
        return h->status;
    return check_device(h);
}
}  // namespace

int pic_load_profiles(pic_handle* h, int32_t n_points, const double* n_e, const double* n_i,
                      const double* mean_energy_e_eV, const double* flux_i) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (n_points < 2 || n_points > 65536) return fail(h, PIC_EINVAL, "n_points must be in [2, 65536]");
    pic::Ctrl c;
    if (check_profiles(h, n_points, n_e, n_i, mean_energy_e_eV, flux_i, &c)) return h->status;
    std::vector<double> tab((size_t)8 * n_points);
    int64_t count[2];
    for (int s = 0; s < 2; ++s)
        if (profile_table(h, s, n_points, n_e, n_i, mean_energy_e_eV, flux_i, tab.data() + (size_t)4 * n_points * s,
                          &count[s]))
            return h->status;
    double* dtab = nullptr;
    if (!hip_ok(h, hipMalloc(&dtab, sizeof(double) * tab.size()), "hipMalloc")) return h->status;
    int rc = hip_ok(h, hipMemcpyAsync(dtab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, h->stream),
                    "copy profiles")
                 ? load_from_tables(h, c, n_points, dtab, count)
                 : h->status;
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(dtab);
    return rc ? rc : h->status;
}

int pic_load_profiles_noalloc(pic_handle* h, int32_t n_points, const double* n_e, const double* n_i,
                              const double* mean_energy_e_eV, const double* flux_i) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (n_points < 2 || n_points > PIC_NOALLOC_MAX_POINTS)
        return fail(h, PIC_EINVAL, "n_points must be in [2, PIC_NOALLOC_MAX_POINTS] for the no-allocation loader");
    int dev = -1;
    if (!hip_ok(h, hipGetDevice(&dev), "hipGetDevice")) return h->status;
    if (dev != h->device) return fail(h, PIC_EINVAL, "the handle's device must be current");
    double* dtab = nullptr;
    size_t room = 0;
    if (!hip_ok(h, pic::noalloc_scratch(dev, &dtab, &room), "scratch address")) return h->status;
    if ((size_t)8 * n_points > room) return fail(h, PIC_EINVAL, "profiles exceed the no-allocation staging");
    pic::Ctrl c;
    if (check_profiles(h, n_points, n_e, n_i, mean_energy_e_eV, flux_i, &c)) return h->status;
    // one species at a time through a fixed host buffer: nothing is allocated
    double tab[4 * pic::kNoAllocMaxPoints];
    int64_t count[2];
    for (int s = 0; s < 2; ++s) {
        if (profile_table(h, s, n_points, n_e, n_i, mean_energy_e_eV, flux_i, tab, &count[s])) return h->status;
        if (!hip_ok(h, hipMemcpyAsync(dtab + (size_t)4 * n_points * s, tab, sizeof(double) * 4 * n_points,
                                      hipMemcpyHostToDevice, h->stream),
                    "copy profiles") ||
            !hip_ok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize"))
            return h->status;
    }
    return load_from_tables(h, c, n_points, dtab, count);
}

int pic_diag_config(pic_handle* h, int32_t n_bins, double u_max_eV) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (n_bins < 1 || n_bins > 4096) return fail(h, PIC_EINVAL, "n_bins must be in [1, 4096]");
    if (!(u_max_eV > 0.0) || !std::isfinite(u_max_eV)) return fail(h, PIC_EINVAL, "u_max_eV must be finite and > 0");
    if (check_device(h)) return h->status;
    const int nn = h->cfg.n_cells + 1;
    const size_t lds = pic::diag_lds_bytes(nn, n_bins);
    if (lds > 160 * 1024) return fail(h, PIC_EINVAL, "n_cells and n_bins need more than 160 KiB of LDS");
    pic::DiagDev& D = h->diag;
    if (!D.node) {
        if (!dev_alloc(h, &D.node, (size_t)8 * nn) || !dev_alloc(h, &D.fx_sample, (size_t)nn) ||
            !dev_alloc(h, &D.counts, 2))
            return h->status;
    }
    if (n_bins > h->diag_capacity_bins) {
        if (!dev_alloc(h, &D.hist, (size_t)n_bins)) return h->status;
        h->diag_capacity_bins = n_bins;
    }
    D.n_bins = n_bins;
    D.bins_per_eV = (float)(n_bins / u_max_eV);
    D.e0 = kE0;
    D.n_iz = 0;
    for (int k = 0; k < h->P.sp_n[0]; ++k)
        if (h->P.proc[0][k].kind == PIC_E_IONIZATION) D.iz[D.n_iz++] = k;
    h->diag_umax = u_max_eV;
    if (!hip_ok(h, pic::set_diag_lds_limit(lds), "hipFuncSetAttribute") ||
        !hip_ok(h, hipMemsetAsync(D.node, 0, sizeof(double) * 8 * nn, h->stream), "zero diagnostics") ||
        !hip_ok(h, hipMemsetAsync(D.fx_sample, 0, sizeof(double) * nn, h->stream), "zero diagnostics") ||
        !hip_ok(h, hipMemsetAsync(D.hist, 0, sizeof(unsigned long long) * n_bins, h->stream), "zero diagnostics") ||
        !hip_ok(h, hipMemsetAsync(D.counts, 0, sizeof(unsigned long long) * 2, h->stream), "zero diagnostics"))
        return h->status;
    return check_device(h);
}

int pic_diag_sample(pic_handle* h) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (!h->diag.node) return fail(h, PIC_ESTATE, "pic_diag_config was not called");
    if (complete_pending(h)) return h->status;
    const int blocks = (int)std::min<int64_t>(512, std::max<int64_t>(1, (h->cfg.capacity[0] + 255) / 256));
    if (!hip_ok(h, pic::launch_diag(h->P, h->diag, blocks, h->stream), "diag launch")) return h->status;
    return PIC_OK;
}

int pic_diag_read(pic_handle* h, pic_diag_out* out, int reset) {
    if (!h || !out) return h ? fail(h, PIC_EINVAL, "out is NULL") : PIC_EINVAL;
    if (h->status) return h->status;
    if (!h->diag.node) return fail(h, PIC_ESTATE, "pic_diag_config was not called");
    const int nn = h->cfg.n_cells + 1, nb = h->diag.n_bins;
    if (out->n_nodes != nn) return fail(h, PIC_EINVAL, "out->n_nodes must be n_cells + 1");
    if (out->eedf_eV_m32 && out->n_bins != nb) return fail(h, PIC_EINVAL, "out->n_bins must be the configured n_bins");
    if (check_device(h)) return h->status;
    std::vector<double> node((size_t)8 * nn);
    std::vector<unsigned long long> hist((size_t)nb), counts(2);
    if (!hip_ok(h, hipMemcpy(node.data(), h->diag.node, sizeof(double) * node.size(), hipMemcpyDeviceToHost), "copy") ||
        !hip_ok(h, hipMemcpy(hist.data(), h->diag.hist, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost), "copy") ||
        !hip_ok(h, hipMemcpy(counts.data(), h->diag.counts, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost),
                "copy"))
        return h->status;
    const double ns = (double)std::max<unsigned long long>(counts[1], 1);
    const double* n = node.data();
    for (int i = 0; i < nn; ++i) {
        const double V = (i == 0 || i == nn - 1) ? 0.5 * h->dx : h->dx;
        const double f = h->W / (V * ns);
        if (out->n_e_m3) out->n_e_m3[i] = f * n[i];
        if (out->mean_energy_e_eV) out->mean_energy_e_eV[i] = n[i] > 0.0 ? n[nn + i] / n[i] : std::nan("");
        if (out->energy_flux_e_W_m2) out->energy_flux_e_W_m2[i] = f * n[2 * nn + i];
        if (out->ionisation_rate_m3s) out->ionisation_rate_m3s[i] = f * n[3 * nn + i];
        if (out->n_fast_m3) out->n_fast_m3[i] = f * n[4 * nn + i];
        if (out->flux_e_m2s) out->flux_e_m2s[i] = f * n[5 * nn + i];
        if (out->heating_W_m3) out->heating_W_m3[i] = f * n[6 * nn + i];
        if (out->E_V_m) out->E_V_m[i] = n[7 * nn + i] / ns;
    }
    const double du = h->diag_umax / nb, ne = (double)std::max<unsigned long long>(counts[0], 1);
    if (out->eedf_eV_m32)
        for (int k = 0; k < nb; ++k) out->eedf_eV_m32[k] = (double)hist[k] / (ne * du * std::sqrt((k + 0.5) * du));
    out->n_samples = (int64_t)counts[1];
    out->n_electrons = (int64_t)counts[0];
    out->u_max_eV = h->diag_umax;
    if (reset && (!hip_ok(h, hipMemset(h->diag.node, 0, sizeof(double) * 8 * nn), "zero diagnostics") ||
                  !hip_ok(h, hipMemset(h->diag.hist, 0, sizeof(unsigned long long) * nb), "zero diagnostics") ||
                  !hip_ok(h, hipMemset(h->diag.counts, 0, sizeof(unsigned long long) * 2), "zero diagnostics")))
        return h->status;
    return PIC_OK;
}

int pic_electrode_fluxes(pic_handle* h, int32_t n, double* gamma_e, double* gamma_i) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (n != h->spp || !gamma_e || !gamma_i)
        return fail(h, PIC_EINVAL, "n must be the steps per RF period and the arrays non-NULL");
    if (check_device(h)) return h->status;
    std::vector<unsigned long long> t((size_t)2 * n);
    if (!hip_ok(h, hipMemcpy(t.data(), h->P.flux_trace, sizeof(unsigned long long) * t.size(), hipMemcpyDeviceToHost),
                "copy flux trace"))
        return h->status;
    const double f = h->W / h->cfg.dt_s;
    for (int k = 0; k < n; ++k) {
        gamma_e[k] = f * (double)t[2 * k];
        gamma_i[k] = f * (double)t[2 * k + 1];
    }
    return PIC_OK;
}

int pic_get_fields(pic_handle* h, double* q_nodes, double* phi, float* e_nodes) {
    if (!h) return PIC_EINVAL;
    if (check_device(h)) return h->status;
    const size_t nn = (size_t)h->cfg.n_cells + 1;
    if (q_nodes && !hip_ok(h, hipMemcpy(q_nodes, h->P.Q_last, nn * 8, hipMemcpyDeviceToHost), "copy Q")) return h->status;
    if (phi && !hip_ok(h, hipMemcpy(phi, h->P.phi, nn * 8, hipMemcpyDeviceToHost), "copy phi")) return h->status;
    if (e_nodes && !hip_ok(h, hipMemcpy(e_nodes, h->P.E, nn * 4, hipMemcpyDeviceToHost), "copy E")) return h->status;
    return PIC_OK;
}

int pic_set_record_decisions(pic_handle* h, int on) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (check_device(h)) return h->status;
    for (int s = 0; s < 2; ++s) {
        if (on && !h->dec_store[s]) {
            if (!dev_alloc(h, &h->dec_store[s], (size_t)h->cfg.capacity[s])) return h->status;
            if (!hip_ok(h, hipMemset(h->dec_store[s], 0, (size_t)h->cfg.capacity[s]), "zero decisions")) return h->status;
        }
        h->P.dec[s] = on ? h->dec_store[s] : nullptr;
    }
    drop_graph(h);   // the captured launches carry the old parameters
    return PIC_OK;
}

int pic_get_decisions(pic_handle* h, int species, uint32_t* id, int8_t* code, int64_t capacity, int64_t* n_out) {
    if (!h || !n_out) return h ? fail(h, PIC_EINVAL, "n_out is NULL") : PIC_EINVAL;
    if (h->status) return h->status;
    if (species != 0 && species != 1) return fail(h, PIC_EINVAL, "species must be 0 or 1");
    if (!h->dec_store[species]) return fail(h, PIC_ESTATE, "decision recording was never enabled");
    if (check_device(h)) return h->status;
    pic::Ctrl c;
    if (read_ctrl(h, &c)) return h->status;
    const int64_t ns = c.n_slots[species];
    const unsigned b = c.cur;
    std::vector<float> hx(ns);
    std::vector<uint32_t> hid(ns);
    std::vector<int8_t> hd(ns);
    if (ns > 0 &&
        (!hip_ok(h, hipMemcpy(hx.data(), h->P.x[b][species], ns * 4, hipMemcpyDeviceToHost), "copy x") ||
         !hip_ok(h, hipMemcpy(hid.data(), h->P.id[b][species], ns * 4, hipMemcpyDeviceToHost), "copy id") ||
         !hip_ok(h, hipMemcpy(hd.data(), h->dec_store[species], ns, hipMemcpyDeviceToHost), "copy decisions")))
        return h->status;
    int64_t n = 0;
    for (int64_t i = 0; i < ns; ++i) n += hx[i] > 0.0f;
    *n_out = n;
    if (!id && !code) return PIC_OK;
    if (capacity < n) return fail(h, PIC_EINVAL, "capacity too small");
    int64_t k = 0;
    for (int64_t i = 0; i < ns; ++i) {
        if (!(hx[i] > 0.0f)) continue;
        if (id) id[k] = hid[i];
        if (code) code[k] = hd[i];
        ++k;
    }
    return PIC_OK;
}

int pic_timing(pic_handle* h, int start, double* mean_ms, int64_t* n_launches) {
    if (!h) return PIC_EINVAL;
    if (h->status) return h->status;
    if (start) {
        if (check_device(h)) return h->status;
        h->timing = true;
        h->n_timed = 0;
        return PIC_OK;
    }
    if (check_device(h)) return h->status;
    double sum = 0.0;
    for (int64_t k = 0; k < h->n_timed; ++k) {
        float ms = 0.0f;
        if (!hip_ok(h, hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]), "hipEventElapsedTime"))
            return h->status;
        sum += ms;
    }
    if (mean_ms) *mean_ms = h->n_timed ? sum / (double)h->n_timed : 0.0;
    if (n_launches) *n_launches = h->n_timed;
    h->timing = false;
    return PIC_OK;
}


// ---------------------------------------------------------------------------------------
// Batches of discharges
// ---------------------------------------------------------------------------------------
struct pic_batch {
    std::vector<pic_handle*> hs;
    hipStream_t stream = nullptr;
    pic::Params* dparams = nullptr;
    int* dseg = nullptr;
    std::vector<int> seg;   // workgroup offsets, n + 1 entries
    int threads = 256;
    size_t lds = 0;
    double rounds = 4.0;   // workgroups per launch in units of the device's resident workgroups
    int status = PIC_OK;
    std::string err;
    // timing of the batched particle pass
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int64_t n_timed = 0;
    // reordering of all discharges in one launch per stage: block offsets (n + 1 entries)
    std::vector<int> sseg;
    int* dsseg = nullptr;
    int max_cells = 1;
    // captured graph of graph_steps steps; valid from the per-discharge reorder phases gsig
    // (steps since the last reordering) and pending state gpend; it advances the phases to
    // gend and leaves every discharge's last step pending
    int64_t graph_steps = 0;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> gsig, gend;
    bool gpend = false;
    hipStream_t cap = nullptr;   // private stream the graph is captured on
    int64_t graph_launches = 0;
    bool record = false;         // batched launches write the decision records (test hook)
};

namespace {
thread_local std::string g_batch_error;

int bfail(pic_batch* b, int code, const std::string& msg) {
    if (!b) {
        g_batch_error = msg;
        return code;
    }
    if (b->status == PIC_OK) {
        b->status = code;
        b->err = msg;
    }
    return b->status;
}

// first error of any discharge, with its index
int batch_status(pic_batch* b) {
    if (b->status) return b->status;
    for (size_t k = 0; k < b->hs.size(); ++k)
        if (b->hs[k]->status)
            return bfail(b, b->hs[k]->status, "discharge " + std::to_string(k) + ": " + b->hs[k]->err);
    return PIC_OK;
}

// Brings every discharge to the same pending state: completes, one by one, the pending
// steps of a batch whose discharges disagree (per-discharge queries complete theirs).
int batch_align(pic_batch* b) {
    bool any = false, all = true;
    for (pic_handle* h : b->hs) {
        any |= h->pending;
        all &= h->pending;
    }
    if (any && !all)
        for (pic_handle* h : b->hs)
            if (h->pending && complete_pending(h)) break;
    return batch_status(b);
}

int batch_launch(pic_batch* b, int mode) {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (b->timing && (mode & pic::kAdvance)) {
        const size_t k = (size_t)b->n_timed * 2;
        if (k + 2 > b->ev.size()) {
            if (b->ev.size() >= 2 * 8192) {
                b->timing = false;
            } else {
                for (int q = 0; q < 2; ++q) {
                    hipEvent_t e;
                    if (hipEventCreate(&e) != hipSuccess) return bfail(b, PIC_EHIP, "hipEventCreate");
                    b->ev.push_back(e);
                }
            }
        }
        if (b->timing) {
            ea = b->ev[k];
            eb = b->ev[k + 1];
            if (hipEventRecord(ea, b->stream) != hipSuccess) return bfail(b, PIC_EHIP, "hipEventRecord");
        }
    }
    const int m = mode | ((b->record && (mode & pic::kComplete)) ? pic::kRecord : 0);
    const hipError_t e = pic::launch_pass_batch(m, b->dparams, b->dseg, (int)b->hs.size(), b->seg.back(),
                                                b->threads, b->lds, b->stream);
    if (e != hipSuccess) return bfail(b, PIC_EHIP, std::string("batched pass launch: ") + hipGetErrorString(e));
    if (eb) {
        if (hipEventRecord(eb, b->stream) != hipSuccess) return bfail(b, PIC_EHIP, "hipEventRecord");
        ++b->n_timed;
    }
    return PIC_OK;
}
// Launch shape of the batched pass: blockDim `threads` (every discharge's n_cells + 1 must
// be <= 8 threads), and about `rounds` x the workgroups resident on the device at once,
// split over the discharges in proportion to the weights w (their particles); each
// discharge gets at least 2 and at most one per 4 x blockDim particles.  Uploads the block
// offsets when the device table exists.
hipError_t batch_layout(pic_batch* b, int threads, double rounds, const std::vector<double>& w) {
    size_t lds = 0;
    for (pic_handle* h : b->hs) lds = std::max(lds, pass_lds_bytes(h->cfg.n_cells + 1, threads));
    hipError_t e = pic::set_pass_batch_lds_limit(lds);
    int cus = 0, per_cu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->hs[0]->device);
    if (e == hipSuccess) e = pic::pass_batch_occupancy(threads, lds, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    double total = 0.0;
    for (double x : w) total += x;
    const double resident = rounds * (double)cus * (double)per_cu;
    std::vector<int> seg(1, 0);
    for (size_t k = 0; k < b->hs.size(); ++k) {
        const int cap = std::max(2, (int)std::ceil(w[k] / (4.0 * threads)));
        const int g = std::min(cap, std::max(2, (int)std::lround(resident * w[k] / std::max(total, 1.0))));
        seg.push_back(seg.back() + g);
    }
    if (b->dseg) {
        e = hipMemcpy(b->dseg, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
    }
    b->threads = threads;
    b->lds = lds;
    b->rounds = rounds;
    b->seg = seg;
    return hipSuccess;
}
}  // namespace

void pic_batch_free(pic_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (pic_handle* h : b->hs) pic_free(h);
    if (b->dparams) (void)hipFree(b->dparams);
    if (b->dseg) (void)hipFree(b->dseg);
    if (b->dsseg) (void)hipFree(b->dsseg);
    delete b;
}

int pic_batch_init(const pic_config* cfgs, int n, void* hip_stream, pic_batch** out) {
    if (!out) return bfail(nullptr, PIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs) return bfail(nullptr, PIC_EINVAL, "cfgs is NULL");
    if (n < 1 || n > 4096) return bfail(nullptr, PIC_EINVAL, "n must be in [1, 4096]");
    for (int k = 0; k < n; ++k) {   // every configuration is checked before any device work
        const std::string bad = validate(&cfgs[k]);
        if (!bad.empty()) return bfail(nullptr, PIC_EINVAL, "discharge " + std::to_string(k) + ": " + bad);
    }
    pic_batch* b = new (std::nothrow) pic_batch();
    if (!b) return bfail(nullptr, PIC_ENOMEM, "out of host memory");
    b->stream = static_cast<hipStream_t>(hip_stream);
    int max_nn = 0;
    for (int k = 0; k < n; ++k) {
        pic_handle* h = nullptr;
        const int rc = pic_init(&cfgs[k], hip_stream, &h);
        if (rc) {
            const std::string msg = "discharge " + std::to_string(k) + ": " + g_init_error;
            pic_batch_free(b);
            return bfail(nullptr, rc, msg);
        }
        b->hs.push_back(h);
        max_nn = std::max(max_nn, cfgs[k].n_cells + 1);
    }
    // One workgroup size for the launch (the epilogue needs n_cells + 1 <= 8 x blockDim), and
    // about four resident rounds of workgroups: the discharges' uneven costs then even out
    // in the hardware's dispatch (measured on a 64-discharge sweep: 1.32 ms per launch with
    // one round, 0.97 ms with four).  pic_batch_autotune revises both.
    {
        std::vector<double> w;
        for (int k = 0; k < n; ++k) w.push_back((double)(cfgs[k].n_init_super[0] + cfgs[k].n_init_super[1]));
        const hipError_t e = batch_layout(b, max_nn <= 2048 ? 256 : 1024, 4.0, w);
        if (e != hipSuccess) {
            const std::string msg = std::string("batch set-up: ") + hipGetErrorString(e);
            pic_batch_free(b);
            return bfail(nullptr, PIC_EHIP, msg);
        }
    }
    hipError_t e = hipSuccess;
    // reordering blocks: each discharge keeps its own count
    b->sseg.assign(1, 0);
    for (int k = 0; k < n; ++k) {
        b->sseg.push_back(b->sseg.back() + b->hs[k]->sort_blocks);
        b->max_cells = std::max(b->max_cells, cfgs[k].n_cells);
    }
    std::vector<pic::Params> hp(n);
    for (int k = 0; k < n; ++k) hp[k] = b->hs[k]->P;
    if ((e = hipMalloc(&b->dparams, sizeof(pic::Params) * n)) != hipSuccess ||
        (e = hipMalloc(&b->dseg, sizeof(int) * (n + 1))) != hipSuccess ||
        (e = hipMalloc(&b->dsseg, sizeof(int) * (n + 1))) != hipSuccess ||
        (e = hipMemcpy(b->dparams, hp.data(), sizeof(pic::Params) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->dseg, b->seg.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->dsseg, b->sseg.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice)) != hipSuccess) {
        const std::string msg = std::string("batch set-up: ") + hipGetErrorString(e);
        pic_batch_free(b);
        return bfail(nullptr, e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EHIP, msg);
    }
    *out = b;
    return PIC_OK;
}

namespace {
// One batched step: the particle pass of every discharge, then the reorderings that are
// due (in one launch per stage when every discharge is due, else one by one).
int batch_one_step(pic_batch* b) {
    const int mode = pic::kAdvance | (b->hs[0]->pending ? pic::kComplete : 0);
    if (batch_launch(b, mode)) return b->status;
    size_t due = 0;
    for (pic_handle* h : b->hs) {
        h->pending = true;
        if (h->cfg.sort_every > 0 && h->since_sort + 1 >= h->cfg.sort_every) ++due;
    }
    if (due == b->hs.size()) {
        const hipError_t e = pic::launch_sort_batch(b->dparams, b->dsseg, (int)b->hs.size(), b->sseg.back(),
                                                    b->max_cells, b->stream);
        if (e != hipSuccess) return bfail(b, PIC_EHIP, std::string("batched sort launch: ") + hipGetErrorString(e));
        for (pic_handle* h : b->hs) h->since_sort = 0;
        return PIC_OK;
    }
    for (pic_handle* h : b->hs) {
        if (h->cfg.sort_every > 0 && ++h->since_sort >= h->cfg.sort_every) {
            if (!hip_ok(h, pic::launch_sort(h->P, h->sort_cnt, h->sort_cursor, h->sort_blocks, h->sort_threads,
                                            h->stream),
                        "sort launch"))
                return batch_status(b);
            h->since_sort = 0;
        }
    }
    return PIC_OK;
}

std::vector<int> batch_phases(const pic_batch* b) {
    std::vector<int> v;
    for (const pic_handle* h : b->hs) v.push_back(h->since_sort);
    return v;
}

// Records graph_steps batched steps, starting from the current reorder phases and pending
// state (the same for every discharge), into a graph on a private stream.  Nothing runs;
// the host-side phases and pending flags are put back.
int batch_capture(pic_batch* b) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bfail(b, PIC_EHIP, "hipStreamCreateWithFlags");
    const std::vector<int> sig = batch_phases(b);
    const bool pend = b->hs[0]->pending;
    const hipStream_t user = b->stream;
    const bool timing = b->timing;
    b->timing = false;
    b->stream = b->cap;
    for (pic_handle* h : b->hs) h->stream = b->cap;
    hipGraph_t g = nullptr;
    int rc = PIC_OK;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        rc = bfail(b, PIC_EHIP, "hipStreamBeginCapture");
    } else {
        for (int64_t k = 0; k < b->graph_steps && rc == PIC_OK; ++k) rc = batch_one_step(b);
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc == PIC_OK && e != hipSuccess) rc = bfail(b, PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    b->gend = batch_phases(b);
    for (size_t k = 0; k < b->hs.size(); ++k) {
        b->hs[k]->since_sort = sig[k];
        b->hs[k]->pending = pend;
        b->hs[k]->stream = user;
    }
    b->stream = user;
    b->timing = timing;
    if (rc == PIC_OK) {
        const hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            rc = bfail(b, PIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc == PIC_OK) {
        b->gsig = sig;
        b->gpend = pend;
    }
    return rc;
}
}  // namespace

int pic_batch_step(pic_batch* b, int64_t n_steps) {
    if (!b) return PIC_EINVAL;
    if (batch_status(b)) return b->status;
    if (n_steps < 0) return bfail(b, PIC_EINVAL, "n_steps must be >= 0");
    if (n_steps > 0 && batch_align(b)) return b->status;
    int64_t k = 0;
    while (k < n_steps) {
        if (b->graph_steps > 0 && n_steps - k >= b->graph_steps && !b->timing) {
            if ((!b->gexec || b->hs[0]->pending != b->gpend || batch_phases(b) != b->gsig) && batch_capture(b))
                return b->status;
            if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return bfail(b, PIC_EHIP, "hipGraphLaunch");
            for (size_t q = 0; q < b->hs.size(); ++q) {
                b->hs[q]->since_sort = b->gend[q];
                b->hs[q]->pending = true;
            }
            ++b->graph_launches;
            k += b->graph_steps;
            continue;
        }
        if (batch_one_step(b)) return b->status;
        ++k;
    }
    return PIC_OK;
}

int pic_batch_set_graph(pic_batch* b, int64_t steps_per_graph) {
    if (!b) return PIC_EINVAL;
    if (batch_status(b)) return b->status;
    if (steps_per_graph < 0 || steps_per_graph > 100000)
        return bfail(b, PIC_EINVAL, "steps_per_graph must be in [0, 100000]");
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, PIC_EHIP, "hipStreamSynchronize");
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->graph_steps = steps_per_graph;
    b->graph_launches = 0;
    return PIC_OK;
}

int pic_batch_rebalance(pic_batch* b) {
    if (!b) return PIC_EINVAL;
    if (pic_batch_sync(b)) return b->status;
    std::vector<double> w;
    for (pic_handle* h : b->hs) {
        pic::Ctrl c;
        if (read_ctrl(h, &c)) return batch_status(b);
        w.push_back((double)std::max<int64_t>(1, c.n_alive[0] + c.n_alive[1]));
    }
    if (b->gexec) {   // the launch shape changes
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    const hipError_t e = batch_layout(b, b->threads, b->rounds, w);
    if (e != hipSuccess) return bfail(b, PIC_EHIP, std::string("batch layout: ") + hipGetErrorString(e));
    return PIC_OK;
}

int pic_batch_set_record_decisions(pic_batch* b, int on) {
    if (!b) return PIC_EINVAL;
    if (pic_batch_sync(b)) return b->status;
    for (pic_handle* h : b->hs)
        if (pic_set_record_decisions(h, on)) return batch_status(b);
    std::vector<pic::Params> hp;
    for (pic_handle* h : b->hs) hp.push_back(h->P);
    if (hipMemcpy(b->dparams, hp.data(), sizeof(pic::Params) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, PIC_EHIP, "parameter upload");
    if (b->gexec) {   // the captured launches carry the old mode
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->record = on != 0;
    return PIC_OK;
}

int pic_batch_graph_launches(const pic_batch* b, int64_t* n) {
    if (!b || !n) return PIC_EINVAL;
    *n = b->graph_launches;
    return PIC_OK;
}

namespace {
struct Tune {
    int threads;
    double rounds;
    int sort_every;
    int order;   // electrons: 1 sorted by cell, 0 compacted in order, -1 each discharge's own choice
};

int batch_apply(pic_batch* b, const Tune& t, const std::vector<double>& w, const std::vector<int>& own) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (t.threads != b->threads || t.rounds != b->rounds) {
        const hipError_t e = batch_layout(b, t.threads, t.rounds, w);
        if (e != hipSuccess) return bfail(b, PIC_EHIP, std::string("batch layout: ") + hipGetErrorString(e));
    }
    bool reload = false;
    for (size_t k = 0; k < b->hs.size(); ++k) {
        pic_handle* h = b->hs[k];
        h->cfg.sort_every = t.sort_every;
        const int order = t.order < 0 ? own[k] : t.order;
        if (h->P.sort_cells[0] != order) {
            h->P.sort_cells[0] = order;
            reload = true;
        }
    }
    if (reload) {
        std::vector<pic::Params> hp;
        for (pic_handle* h : b->hs) hp.push_back(h->P);
        if (hipMemcpy(b->dparams, hp.data(), sizeof(pic::Params) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bfail(b, PIC_EHIP, "parameter upload");
    }
    return PIC_OK;
}

// Mean time per step of `steps` eager batched steps (reorderings included), after two
// untimed steps; steps is a multiple of the reordering interval.
int batch_trial(pic_batch* b, int64_t steps, double* ms) {
    for (int k = 0; k < 2; ++k)
        if (batch_one_step(b)) return b->status;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bfail(b, PIC_EHIP, "hipEventCreate");
    }
    int rc = hipEventRecord(e0, b->stream) == hipSuccess ? PIC_OK : bfail(b, PIC_EHIP, "hipEventRecord");
    for (int64_t k = 0; k < steps && rc == PIC_OK; ++k) rc = batch_one_step(b);
    if (rc == PIC_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = bfail(b, PIC_EHIP, "hipEventRecord");
    if (rc == PIC_OK && hipEventSynchronize(e1) != hipSuccess) rc = bfail(b, PIC_EHIP, "hipEventSynchronize");
    float t = 0.0f;
    if (rc == PIC_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = bfail(b, PIC_EHIP, "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == PIC_OK) {
        for (pic_handle* h : b->hs) check_device(h);
        rc = batch_status(b);
    }
    *ms = (double)t / (double)steps;
    return rc;
}
}  // namespace

int pic_batch_autotune(pic_batch* b, int64_t steps_per_trial, pic_tuning* out) {
    if (!b) return PIC_EINVAL;
    if (batch_status(b)) return b->status;
    if (steps_per_trial < 4 || steps_per_trial > 100000)
        return bfail(b, PIC_EINVAL, "steps_per_trial must be in [4, 100000]");
    if (pic_batch_sync(b)) return b->status;
    // weights of the layout: the particles alive now
    std::vector<double> w;
    int max_nn = 0;
    for (pic_handle* h : b->hs) {
        pic::Ctrl c;
        if (read_ctrl(h, &c)) return batch_status(b);
        w.push_back((double)std::max<int64_t>(1, c.n_alive[0] + c.n_alive[1]));
        max_nn = std::max(max_nn, h->cfg.n_cells + 1);
    }
    int se0 = 0;
    std::vector<int> own;
    for (pic_handle* h : b->hs) {
        if (h->cfg.sort_every <= 0 || h->P.x[1][0] == nullptr)
            return bfail(b, PIC_EINVAL, "autotuning needs every discharge created with sort_every > 0");
        se0 = std::max(se0, h->cfg.sort_every);
        own.push_back(h->P.sort_cells[0]);
    }
    Tune best{b->threads, b->rounds, se0, -1};
    double best_ms = 0.0;
    int trials = 0;
    auto run = [&](const Tune& t, double* ms) -> int {
        if (batch_apply(b, t, w, own)) return b->status;
        const int64_t steps = ((std::max<int64_t>(steps_per_trial, 2 * t.sort_every) + t.sort_every - 1) / t.sort_every) *
                              t.sort_every;
        ++trials;
        return batch_trial(b, steps, ms);
    };
    if (run(best, &best_ms)) return b->status;
    auto consider = [&](Tune t) -> int {
        double ms = 0.0;
        if (run(t, &ms)) return b->status;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
        return PIC_OK;
    };
    // coordinate search: launch size, workgroup size, reordering interval, electron order
    for (double r : {1.0, 2.0, 4.0, 8.0})
        if (r != best.rounds && consider(Tune{best.threads, r, best.sort_every, best.order})) return b->status;
    for (int nt : {256, 512, 1024})
        if (nt != best.threads && max_nn <= 8 * nt && consider(Tune{nt, best.rounds, best.sort_every, best.order}))
            return b->status;
    for (int se : {5, 10, 20, 40, 80})
        if (se != best.sort_every && consider(Tune{best.threads, best.rounds, se, best.order})) return b->status;
    for (int order : {0, 1})
        if (consider(Tune{best.threads, best.rounds, best.sort_every, order})) return b->status;
    if (batch_apply(b, best, w, own)) return b->status;
    if (out) {
        out->threads = best.threads;
        out->sort_every = best.sort_every;
        out->electron_order = best.order;
        out->trials = trials;
        out->rounds = best.rounds;
        out->ms_per_step = best_ms;
    }
    return PIC_OK;
}

int pic_batch_sync(pic_batch* b) {
    if (!b) return PIC_EINVAL;
    if (batch_status(b)) return b->status;
    if (batch_align(b)) return b->status;
    if (b->hs[0]->pending) {
        if (batch_launch(b, pic::kComplete)) return b->status;
        for (pic_handle* h : b->hs) h->pending = false;
    }
    for (pic_handle* h : b->hs) check_device(h);
    return batch_status(b);
}

int pic_batch_handle(pic_batch* b, int k, pic_handle** h) {
    if (!b || !h) return PIC_EINVAL;
    if (k < 0 || k >= (int)b->hs.size()) return bfail(b, PIC_EINVAL, "k out of range");
    *h = b->hs[k];
    return PIC_OK;
}

int pic_batch_blocks(const pic_batch* b, int k, int* blocks) {
    if (!b || !blocks || k < 0 || k >= (int)b->hs.size()) return PIC_EINVAL;
    *blocks = b->seg[k + 1] - b->seg[k];
    return PIC_OK;
}

int pic_batch_timing(pic_batch* b, int start, double* mean_ms, int64_t* n_launches) {
    if (!b) return PIC_EINVAL;
    if (batch_status(b)) return b->status;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, PIC_EHIP, "hipStreamSynchronize");
    if (start) {
        b->timing = true;
        b->n_timed = 0;
        return PIC_OK;
    }
    double sum = 0.0;
    for (int64_t k = 0; k < b->n_timed; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, b->ev[2 * k], b->ev[2 * k + 1]) != hipSuccess)
            return bfail(b, PIC_EHIP, "hipEventElapsedTime");
        sum += ms;
    }
    if (mean_ms) *mean_ms = b->n_timed ? sum / (double)b->n_timed : 0.0;
    if (n_launches) *n_launches = b->n_timed;
    b->timing = false;
    return PIC_OK;
}

const char* pic_batch_last_error(const pic_batch* b) {
    if (!b) return g_batch_error.c_str();
    return b->err.c_str();
}

}  // extern "C"
