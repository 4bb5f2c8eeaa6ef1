// gfx950 kernels of the 1D3V PIC/MCC step (Becker et al., arXiv:1608.04601, Sec. 2.5).
//
// One launch of pass_kernel moves every particle once.  A step of velocity Verlet is
// split at the field solve: the launch for step n finishes step n-1 (second half kick
// with E^n, null-collision MCC, ionisation births, moment sample) and starts step n
// (first half kick with the same E^n, drift, wall absorption, cloud-in-cell deposit).
// The field E^n is gathered once per particle and used for both half kicks.  The last
// workgroup to finish (device-scope counter) solves the FP64 Poisson problem for E^{n+1},
// assigns the ids of the step's ionisation products and does the electrode bookkeeping,
// so a step is one kernel launch.
//
// Particles are FP32 structure-of-arrays streamed once per step with coalesced loads;
// vy, vz are read only by collision candidates (and electrons on moment steps) and
// written only after a real collision.  Deposits go to a workgroup-private FP32 copy of
// the grid in LDS and are flushed to the global grid with one atomic per touched node.
// The charge grid is fixed point (integer weights summing to 2^24 per particle): exact,
// and independent of the order in which lanes and workgroups add to it.
#include <mutex>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pic_types.hpp"

namespace pic {

// ----------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two 32x32->64
// products with the published multipliers; the key advances by the published Weyl
// constants between rounds.  Counter = (particle id, 0, step, (species << 8) | stream).
// ----------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    // The round keys are recomputed at every call (scalar adds) rather than kept live in
    // scalar registers across the particle loop, where registers are scarce.
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

enum Stream : uint32_t { kCollision = 0, kTarget = 1, kScatter = 2, kNewIon = 3, kWarm = 0xFE, kLoad = 0xFF };

// u = ((w >> 9) + 1/2) 2^-23 in (0, 1); exact in FP32.
__device__ __forceinline__ float u01(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }
__device__ __forceinline__ double u01d(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

// Box-Muller pair.
__device__ __forceinline__ void normal2(uint32_t a, uint32_t b, float& z0, float& z1) {
    const float r = sqrtf(-2.0f * logf(u01(a)));
    float sn, cs;
    sincospif(2.0f * u01(b), &sn, &cs);
    z0 = r * cs;
    z1 = r * sn;
}

// Isotropic direction, cos(chi) = 1 - 2 ua, azimuth 2 pi ub; sin(chi) = 2 sqrt(ua (1 - ua)).
__device__ __forceinline__ void iso_dir(uint32_t a, uint32_t b, float& nx, float& ny, float& nz) {
    const float ua = u01(a);
    const float c = 1.0f - 2.0f * ua;
    const float sn = 2.0f * sqrtf(ua * (1.0f - ua));
    float sp, cp;
    sincospif(2.0f * u01(b), &sp, &cp);
    nx = c;
    ny = sn * cp;
    nz = sn * sp;
}

// Cloud-in-cell cell and weight of a position t > 0 in cell units (both exact).
__device__ __forceinline__ void cell_of(float t, int nc, int& j, float& w) {
    j = min((int)t, nc - 1);
    w = t - (float)j;
}

// Deposit of one particle to nodes j, j+1 of its species' grid, in fixed point.
__device__ __forceinline__ void lds_count(unsigned long long* a, int j, float w) {
    const unsigned long long wq = (unsigned long long)__float2int_rn(w * kQScale);   // in [0, 2^24]
    atomicAdd(&a[j], kQOne - wq);
    atomicAdd(&a[j + 1], wq);
}

// The live buffer set is picked with a uniform select: indexing the kernel-argument arrays
// with a run-time value would copy them to private memory.
template <typename T>
__device__ __forceinline__ T* bufsel(T* const (&a)[2][2], unsigned cur, int s) {
    return cur ? a[1][s] : a[0][s];
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Everything one workgroup hands to the last workgroup of a launch travels through
// device-scope atomics (read back with device-scope atomic loads), so publishing it needs
// only the completion of this wave's memory operations, not a release fence: an
// agent-scope release would write back and invalidate the whole L2 of the XCD, once per
// workgroup per step.
__device__ __forceinline__ void wait_memory_complete() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// LDS counter slots of one workgroup
enum : int { kCntAbs = 0, kCntColl = 4, kCntViol = 20, kCntErr = 22, kCntTicks = 23, kCntParts = 25, kCntLast = 31,
             kCntSlots = 32 };
static_assert(kCntAbs == kRepAbs && kCntColl == kRepColl && kCntViol == kRepViol && kCntErr == kRepErr &&
                  kCntTicks == kRepTicks && kCntParts == kRepParts,
              "LDS counter slots and report words line up");

// LDS of one workgroup of the particle pass.  A workgroup handles one species at a time:
// Q holds that species' deposit and M its second moment quantity (electron energy or ion
// v_x), U the electron null-collision bounds.  Collision candidates wait in per-wave
// queues (structure of arrays) until a full wave of them can be processed together.
struct Lds {
    uint32_t* cnt;
    unsigned long long* Q;   // fixed-point deposit
    unsigned long long* M;   // fixed-point second moment quantity
    float* E;
    float* U;                // kNullBins + 1
    // collision candidate queues: the candidate's slot and its state as the stream loaded
    // it (v_x completed), so that the MCC reads nothing back from memory (v_y, v_z of ions,
    // which the stream does not load, excepted)
    uint32_t* qslot;
    uint32_t* qr;            // second Philox word of the collision draw
    float* qvx;              // completed v_x
    float* qx;
    uint32_t* qid;
    float* qvy;              // electrons only
    float* qvz;
    // work distribution: block ids of the workgroup's j-th block, tagged (j << 32 | id), and
    // the count of sub-blocks handed to its waves
    unsigned long long* ring;   // kPassRing
    uint32_t* sub;
};

// After the drift of an ionisation product: absorb at the electrodes (Sec. 2.5, ties
// absorbed) or deposit.  Products arise in electron workgroups: the electron goes to the
// workgroup's grid, the ion straight to the global ion grid.
__device__ __forceinline__ float absorb_or_deposit(const Params& P, const Lds& L, int s, float x) {
    if (x > 0.0f && x < P.ncf) {
        int j;
        float w;
        cell_of(x, P.n_cells, j, w);
        if (s == 0) {
            lds_count(L.Q, j, w);
        } else {
            const unsigned long long wq = (unsigned long long)__float2int_rn(w * kQScale);
            unsigned long long* g = P.Qs + (P.n_cells + 1);
            atomicAdd(&g[j], kQOne - wq);
            atomicAdd(&g[j + 1], wq);
        }
        return x;
    }
    if (x <= 0.0f)
        atomicAdd(&L.cnt[kCntAbs + 2 * s + 0], 1u);
    else if (x >= P.ncf)
        atomicAdd(&L.cnt[kCntAbs + 2 * s + 1], 1u);
    else
        atomicOr(&L.cnt[kCntErr], kErrNumeric);
    return -1.0f;   // hole marker
}

// After the drift, without depositing: returns x, or the hole marker after counting the
// absorption (the caller deposits survivors).
__device__ __forceinline__ float absorb_only(const Params& P, const Lds& L, int s, float x) {
    if (x > 0.0f && x < P.ncf) return x;
    if (x <= 0.0f)
        atomicAdd(&L.cnt[kCntAbs + 2 * s + 0], 1u);
    else if (x >= P.ncf)
        atomicAdd(&L.cnt[kCntAbs + 2 * s + 1], 1u);
    else
        atomicOr(&L.cnt[kCntErr], kErrNumeric);
    return -1.0f;
}

// Second moment quantity a = m2 * mscale of a sample at cell weight w, in fixed point: the
// rounded total st and the right node's share s1.  Any physical sample has |a| < 2^30;
// false for larger (or non-finite) values, which the caller adds to the FP64 sums directly.
__device__ __forceinline__ bool moment_fixed(float a, float w, int& st, int& s1) {
    if (!(fabsf(a) < 0x1p30f)) return false;
    st = __float2int_rn(a);
    s1 = __float2int_rn(a * w);
    return true;
}

__device__ __forceinline__ void moment_fp64(const Params& P, int s, int j, float w, float m2) {
    double* sec = P.mom + (s ? 3 : 2) * (P.n_cells + 1);
    unsafeAtomicAdd(&sec[j], (double)m2 * (1.0 - (double)w));
    unsafeAtomicAdd(&sec[j + 1], (double)m2 * (double)w);
}

// One moment sample of species s added to LDS M at once (t <= 0: none).
__device__ __forceinline__ void moment_direct(const Params& P, const Lds& L, int s, float t, float m2) {
    if (!(t > 0.0f)) return;
    int j;
    float w;
    cell_of(t, P.n_cells, j, w);
    int st, s1;
    if (moment_fixed(m2 * (float)P.mscale[s], w, st, s1)) {
        atomicAdd(&L.M[j], (unsigned long long)(long long)(st - s1));
        atomicAdd(&L.M[j + 1], (unsigned long long)(long long)s1);
    } else {
        moment_fp64(P, s, j, w, m2);
    }
}

// One deposit (t <= 0: none) added to LDS Q at once.
__device__ __forceinline__ void deposit_direct(const Lds& L, int nc, float t) {
    if (!(t > 0.0f)) return;
    int j;
    float w;
    cell_of(t, nc, j, w);
    lds_count(L.Q, j, w);
}

// Per-lane run caches for cell-sorted particles (ions, which move a small fraction of a
// cell per step): a lane's successive particles lie in the same cell most of the time, so
// their contributions are summed in registers and reach LDS once per run.
struct ChargeRun {
    int c = -1;   // cell of the run
    int n = 0;    // particles in it (at most 64, so d stays below 2^31)
    int d = 0;    // sum of right-node weights
};

struct MomentRun {
    int c = -1;
    long long st = 0;   // sum of fixed-point totals
    long long s1 = 0;   // sum of right-node shares
};

__device__ __forceinline__ void flush_run(const Lds& L, ChargeRun& r) {
    if (r.n > 0) {
        atomicAdd(&L.Q[r.c], (unsigned long long)(r.n * (int)kQOne - r.d));
        atomicAdd(&L.Q[r.c + 1], (unsigned long long)r.d);
    }
    r.n = 0;
    r.d = 0;
}

__device__ __forceinline__ void flush_run(const Lds& L, MomentRun& r) {
    if (r.c >= 0) {
        atomicAdd(&L.M[r.c], (unsigned long long)(r.st - r.s1));
        atomicAdd(&L.M[r.c + 1], (unsigned long long)r.s1);
    }
    r.st = 0;
    r.s1 = 0;
}

__device__ __forceinline__ void deposit_run(const Lds& L, int nc, ChargeRun& r, float t) {
    if (!(t > 0.0f)) return;
    int j;
    float w;
    cell_of(t, nc, j, w);
    const int d1 = __float2int_rn(w * kQScale);
    if (j != r.c || r.n == 64) {
        flush_run(L, r);
        r.c = j;
    }
    r.n += 1;
    r.d += d1;
}

__device__ __forceinline__ void moment_run(const Params& P, const Lds& L, int s, MomentRun& r, float t, float m2) {
    if (!(t > 0.0f)) return;
    int j;
    float w;
    cell_of(t, P.n_cells, j, w);
    int st, s1;
    if (!moment_fixed(m2 * (float)P.mscale[s], w, st, s1)) {
        moment_fp64(P, s, j, w, m2);
        return;
    }
    if (j != r.c) {
        flush_run(L, r);
        r.c = j;
    }
    r.st += st;
    r.s1 += s1;
}

// Moment sample of an ionisation product (rare), straight to the FP64 window sums: its
// density weight (the density of all other particles comes from the deposit) and its
// second quantity.
__device__ __forceinline__ void sample_product(const Params& P, int s, float x, float m2) {
    const int nn = P.n_cells + 1;
    int j;
    float w;
    cell_of(x, P.n_cells, j, w);
    double* dens = P.mom + s * nn;
    unsafeAtomicAdd(&dens[j], 1.0 - (double)w);
    unsafeAtomicAdd(&dens[j + 1], (double)w);
    moment_fp64(P, s, j, w, m2);
}

// Products of one ionisation at the parent's position x^n.
template <int MODE>
__device__ __forceinline__ void spawn_products(const Params& P, const Lds& L, float x, float E, float sp, float n2x,
                                            float n2y, float n2z, uint4 D, uint32_t pid, unsigned cur, int64_t ns0,
                                            int64_t ns1, bool sample) {
    float y0, y1, y2, y3;
    normal2(D.x, D.y, y0, y1);
    normal2(D.z, D.w, y2, y3);
    const unsigned k = atomicAdd(&P.ctrl->n_births, 1u);
    if ((int)k < P.max_births && ns0 + (int64_t)k < P.cap[0] && ns1 + (int64_t)k < P.cap[1]) {
        st_agent(&P.birth_parent[k], pid);
        // products at the parent's position x^n with end-of-step velocities
        float cev[3] = {sp * n2x, sp * n2y, sp * n2z};
        float civ[3] = {P.vT * y0, P.vT * y1, P.vT * y2};
        if (sample) {
            sample_product(P, 0, x, P.half_m_over_e[0] * (cev[0] * cev[0] + cev[1] * cev[1] + cev[2] * cev[2]));
            sample_product(P, 1, x, civ[0]);
        }
        float cex = x, cix = x;
        if (MODE & kAdvance) {   // products are moved from the next step on
            cev[0] += P.kick[0] * E;
            civ[0] += P.kick[1] * E;
            cex = absorb_or_deposit(P, L, 0, fmaf(cev[0], P.dt_over_dx, x));
            cix = absorb_or_deposit(P, L, 1, fmaf(civ[0], P.dt_over_dx, x));
        }
        const int64_t se = ns0 + k, si = ns1 + k;
        bufsel(P.x, cur, 0)[se] = cex;
        bufsel(P.vx, cur, 0)[se] = cev[0];
        bufsel(P.vy, cur, 0)[se] = cev[1];
        bufsel(P.vz, cur, 0)[se] = cev[2];
        bufsel(P.x, cur, 1)[si] = cix;
        bufsel(P.vx, cur, 1)[si] = civ[0];
        bufsel(P.vy, cur, 1)[si] = civ[1];
        bufsel(P.vz, cur, 1)[si] = civ[2];
        if (MODE & kRecord) {
            P.dec[0][se] = 0;
            P.dec[1][si] = 0;
        }
    }
}

// Finish a particle whose collision test (if any) is done: moment sample of the end-of-step
// state, first half kick and drift of the next step, absorption.  x and vx become the values
// to store; tq is the position to deposit as charge (<= 0: none) and tm, m2 the position and
// second quantity of the moment sample (tm <= 0: none).
template <int MODE, int S>
__device__ __forceinline__ void finish(const Params& P, const Lds& L, float& x, float& vx, float vy, float vz,
                                       float kE, bool sample, float& tq, float& tm, float& m2) {
    if ((MODE & kComplete) && sample) {
        tm = x;
        m2 = S == 0 ? P.half_m_over_e[0] * (vx * vx + vy * vy + vz * vz) : vx;
    }
    if (MODE & kAdvance) {
        vx += kE;                                  // v^{n+1/2}
        x = absorb_only(P, L, S, fmaf(vx, P.dt_over_dx, x));
        tq = x;
    }
}

// Streaming part for one particle of species S in slot i (x, vx, id and, for electrons on
// completing launches, vy, vz loaded by the caller): gather E^n once, complete the previous
// step's kick, and test for a collision candidate with one integer comparison.  Stores
// nothing: on return x and vx are the values for the caller to store (a hole keeps its
// own).  Non-candidates are finished here; a candidate returns true with x unchanged, its
// completed v_x in vx and the second Philox word in rword, to be queued.
template <int MODE, int S>
__device__ __forceinline__ bool stream_particle(const Params& P, const Lds& L, int64_t i, float& x, float& vx,
                                                uint32_t pid, float vy, float vz, uint32_t stepf, bool sample,
                                                float& tq, float& tm, float& m2, uint32_t& rword) {
    if (!(x > 0.0f)) {   // hole (or a corrupted coordinate)
        if (x != x) atomicOr(&L.cnt[kCntErr], kErrNumeric);
        if (MODE & kRecord) P.dec[S][i] = 0;
        return false;
    }
    if (MODE == kDeposit) {
        tq = x;
        return false;
    }
    int j;
    float w;
    cell_of(x, P.n_cells, j, w);
    const float E = fmaf(w, L.E[j + 1] - L.E[j], L.E[j]);   // cloud-in-cell gather
    const float kE = P.kick[S] * E;                          // half kick, Sec. 2.5 Verlet
    if (MODE & kComplete) {
        vx += kE;   // v^n
        const uint4 A = philox(pid, 0u, stepf, ((uint32_t)S << 8) | kCollision, P.key0, P.key1);
        int8_t code = 0;
        if ((A.x >> 8) < P.T[S]) {   // null-collision candidate
            // Electrons: R nu_max at or above the bound of the summed collision frequency
            // over the particle's g^2 bin means no process can be selected, so the
            // candidate is a null collision without the table lookups (the full test would
            // find the same).
            bool open = true;
            if (S == 0) {
                const float g2 = vx * vx + vy * vy + vz * vz;
                const int b = (int)fminf(g2 * P.inv_gbin, (float)kNullBins);
                open = !(u01(A.y) * P.numax[0] >= L.U[b]);
            }
            if (open) {
                rword = A.y;
                return true;
            }
            code = 1;
        }
        if (MODE & kRecord) P.dec[S][i] = code;
    }
    finish<MODE, S>(P, L, x, vx, vy, vz, kE, sample, tq, tm, m2);
    return false;
}

// Null-collision MCC of queue entry e (Sec. 2.5), then finish it.
template <int MODE, int S>
__device__ __forceinline__ void collide_entry(const Params& P, const Lds& L, unsigned e, uint32_t stepf,
                                              unsigned cur, int64_t ns0, int64_t ns1, bool sample, float& tq,
                                              float& tm, float& m2) {
    const int64_t i = (int64_t)L.qslot[e];
    float vx = L.qvx[e];
    const uint32_t rword = L.qr[e];
    const float x = L.qx[e];
    const uint32_t pid = L.qid[e];
    float vy, vz;
    if (S == 0) {
        vy = L.qvy[e];
        vz = L.qvz[e];
    } else {   // unchanged in memory
        vy = bufsel(P.vy, cur, S)[i];
        vz = bufsel(P.vz, cur, S)[i];
    }
    int j;
    float w;
    cell_of(x, P.n_cells, j, w);
    const float E = fmaf(w, L.E[j + 1] - L.E[j], L.E[j]);
    const float kE = P.kick[S] * E;
    int8_t code = 1;
    bool dirty = false;
    float vtx = 0.0f, vty = 0.0f, vtz = 0.0f;
    if (S == 1) {   // gas atom from the Maxwellian at T_gas
        const uint4 B = philox(pid, 0u, stepf, (1u << 8) | kTarget, P.key0, P.key1);
        float z0, z1, z2, z3;
        normal2(B.x, B.y, z0, z1);
        normal2(B.z, B.w, z2, z3);
        vtx = P.vT * z0;
        vty = P.vT * z1;
        vtz = P.vT * z2;
    }
    const float gx = vx - vtx, gy = vy - vty, gz = vz - vtz;
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float gm = sqrtf(g2);
    const float R = u01(rword) * P.numax[S];
    // n_gas sigma_j [1/m] of the species' processes, four at a time with all their
    // table loads issued before any is used: zero below the threshold, energy raised
    // to the floor emin, the last point at or beyond the table end, linear
    // interpolation in between; selection in config order.  The process table is indexed
    // with compile-time indices only (fully unrolled), and the selected process's kind and
    // threshold are carried in registers.
    float c = 0.0f;
    int sel = -1, skind = -1;
    float sthr = 0.0f;
    const int nsp = P.sp_n[S];
#pragma unroll
    for (int k0 = 0; k0 < kMaxProcPerSpecies; k0 += 4) {
        if (k0 < nsp) {
            float ta[4], tb[4], tf[4];
            bool tbelow[4], ttop[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k0 + k < nsp) {
                    const ProcDev& p = P.proc[S][k0 + k];
                    const float eps = p.efac * g2;
                    const float t = fmaxf(eps, p.emin) * p.inv_de;
                    tbelow[k] = eps < p.thr;
                    ttop[k] = t >= (float)(p.n - 1);
                    const int kk = ttop[k] ? p.n - 2 : (int)t;
                    tf[k] = t - (float)kk;
                    ta[k] = P.tab[p.off + kk];
                    tb[k] = P.tab[p.off + kk + 1];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k0 + k < nsp) {
                    const ProcDev& p = P.proc[S][k0 + k];
                    const float sig = tbelow[k] ? 0.0f : (ttop[k] ? tb[k] : fmaf(tb[k] - ta[k], tf[k], ta[k]));
                    c = fmaf(sig, gm, c);
                    if (sel < 0 && R < c) {
                        sel = p.idx;
                        skind = p.kind;
                        sthr = p.thr;
                    }
                }
            }
        }
    }
    if (c > P.numax[S]) atomicAdd(&L.cnt[kCntViol + S], 1u);
    if (sel >= 0) {
        code = (int8_t)(2 + sel);
        atomicAdd(&L.cnt[kCntColl + sel], 1u);
        const uint4 Cw = philox(pid, 0u, stepf, ((uint32_t)S << 8) | kScatter, P.key0, P.key1);
        float n1x, n1y, n1z;
        iso_dir(Cw.x, Cw.y, n1x, n1y, n1z);
        dirty = true;
        if (skind == 0 || skind == 3) {   // elastic / isotropic: CM-isotropic two-body
            const float fa = P.fa[S], fb = P.fb[S];
            const float sgb = fb * gm;
            vx = fmaf(sgb, n1x, fmaf(fa, vx, fb * vtx));
            vy = fmaf(sgb, n1y, fmaf(fa, vy, fb * vty));
            vz = fmaf(sgb, n1z, fmaf(fa, vz, fb * vtz));
        } else if (S == 0 && skind == 1) {   // excitation: lose the threshold energy
            const float eps = P.half_m_over_e[0] * g2;
            const float sp = sqrtf(fmaxf(eps - sthr, 0.0f) * P.two_e_over_m_e);
            vx = sp * n1x;
            vy = sp * n1y;
            vz = sp * n1z;
        } else if (S == 0 && skind == 2) {   // ionisation: equal share of eps - eps_iz
            const float eps = P.half_m_over_e[0] * g2;
            const float sp = sqrtf(fmaxf(eps - sthr, 0.0f) * P.e_over_m_e);
            vx = sp * n1x;
            vy = sp * n1y;
            vz = sp * n1z;
            float n2x, n2y, n2z;
            iso_dir(Cw.z, Cw.w, n2x, n2y, n2z);
            const uint4 D = philox(pid, 0u, stepf, ((uint32_t)S << 8) | kNewIon, P.key0, P.key1);
            spawn_products<MODE>(P, L, x, E, sp, n2x, n2y, n2z, D, pid, cur, ns0, ns1, sample);
        } else {   // backward: the ion leaves with the atom's velocity
            vx = vtx;
            vy = vty;
            vz = vtz;
        }
    }
    if (MODE & kRecord) P.dec[S][i] = code;
    float xs = x;
    finish<MODE, S>(P, L, xs, vx, vy, vz, kE, sample, tq, tm, m2);
    if (MODE & kAdvance) bufsel(P.x, cur, S)[i] = xs;
    bufsel(P.vx, cur, S)[i] = vx;
    if (dirty) {
        bufsel(P.vy, cur, S)[i] = vy;
        bufsel(P.vz, cur, S)[i] = vz;
    }
}

// Each wave queues its own collision candidates in LDS (kWaveQueue entries) and processes
// them a full wave at a time, so the long MCC path runs on dense waves and the particle
// loop needs no workgroup barrier.  Entries are written and read by the same wave, whose
// LDS operations complete in order; the wavefront fences keep the compiler from moving
// them across each other.
constexpr int kWaveQueue = 128;

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Process queue entries [n - count, n) of this wave, one per lane (count <= 64).
template <int MODE, int S>
__device__ __forceinline__ void drain_queue(const Params& P, const Lds& L, int wq, unsigned n, unsigned count,
                                            uint32_t stepf, unsigned cur, int64_t ns0, int64_t ns1, bool sample) {
    const unsigned lane = threadIdx.x & 63;
    float tq = -1.0f, tm = -1.0f, m2 = 0.0f;
    wave_fence();
    if (lane < count) {
        const unsigned e = wq + n - count + lane;
        collide_entry<MODE, S>(P, L, e, stepf, cur, ns0, ns1, sample, tq, tm, m2);
    }
    deposit_direct(L, P.n_cells, tq);
    if (sample) moment_direct(P, L, S, tm, m2);
    wave_fence();
}

// Registers of one particle as loaded by the stream.
struct Regs {
    float x, vx, vy, vz;
    uint32_t id;
};

template <int MODE, int S>
__device__ __forceinline__ Regs load_particle(const Params& P, unsigned cur, int64_t i) {
    Regs r{-1.0f, 0.0f, 0.0f, 0.0f, 0u};
    r.x = bufsel(P.x, cur, S)[i];
    if (MODE != kDeposit) r.vx = bufsel(P.vx, cur, S)[i];
    if (MODE & kComplete) r.id = bufsel(P.id, cur, S)[i];
    if ((MODE & kComplete) && S == 0) {   // electrons need |v| for the pre-test and the energy
        r.vy = bufsel(P.vy, cur, S)[i];
        r.vz = bufsel(P.vz, cur, S)[i];
    }
    return r;
}

template <int MODE, int S>
__device__ __forceinline__ Regs load_particle_if(const Params& P, unsigned cur, int64_t i, int64_t end) {
    Regs r{-1.0f, 0.0f, 0.0f, 0.0f, 0u};
    if (i < end) r = load_particle<MODE, S>(P, cur, i);
    return r;
}

// Particle i of species S (in range when FULL) with registers r: stream it, store its x and
// vx, deposit, and queue it if it is a collision candidate.
template <int MODE, int S, bool FULL>
__device__ __forceinline__ void process_particle(const Params& P, const Lds& L, int64_t i, int64_t end, Regs r,
                                                 uint32_t stepf, unsigned cur, int64_t ns0, int64_t ns1, bool sample,
                                                 int lane, int wq, ChargeRun& qrun, MomentRun& mrun, unsigned& nq) {
    float tq = -1.0f, tm = -1.0f, m2 = 0.0f;
    uint32_t rw = 0u;
    bool cand = false;
    if (FULL || i < end) {
        cand = stream_particle<MODE, S>(P, L, i, r.x, r.vx, r.id, r.vy, r.vz, stepf, sample, tq, tm, m2, rw);
        if (MODE & kAdvance) bufsel(P.x, cur, S)[i] = r.x;
        if (MODE != kDeposit) bufsel(P.vx, cur, S)[i] = r.vx;
    }
    if (S == 0) {   // electrons leave cell order within a step or two
        deposit_direct(L, P.n_cells, tq);
        if (sample) moment_direct(P, L, S, tm, m2);
    } else {
        deposit_run(L, P.n_cells, qrun, tq);
        if (sample) moment_run(P, L, S, mrun, tm, m2);
    }
    if (MODE & kComplete) {
        const unsigned long long qm = __ballot(cand);
        if (qm) {
            if (cand) {
                const unsigned e = wq + nq + (unsigned)__popcll(qm & ((1ull << lane) - 1ull));
                L.qslot[e] = (uint32_t)i;
                L.qr[e] = rw;
                L.qvx[e] = r.vx;
                L.qx[e] = r.x;
                L.qid[e] = r.id;
                if (S == 0) {
                    L.qvy[e] = r.vy;
                    L.qvz[e] = r.vz;
                }
            }
            nq += (unsigned)__popcll(qm);
            if (nq >= 64u) {
                drain_queue<MODE, S>(P, L, wq, nq, 64u, stepf, cur, ns0, ns1, sample);
                nq -= 64u;
            }
        }
    }
}

// Particles [begin, end) of species S, one per thread per iteration, with the next
// iteration's loads issued before the current particle is processed (one copy of the
// particle code per species keeps the kernel within the instruction cache).  While both the
// current and the next iteration cover every lane, loads and stores are unconditional, so
// the wait for the current particle's data does not also wait for the next one's loads.
template <int MODE, int S>
__device__ __forceinline__ void run_range(const Params& P, const Lds& L, int64_t begin, int64_t end, uint32_t stepf,
                                          unsigned cur, int64_t ns0, int64_t ns1, bool sample) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wq = (tid >> 6) * kWaveQueue;
    ChargeRun qrun;
    MomentRun mrun;
    unsigned nq = 0;   // entries in this wave's queue (wave-uniform)
    const int64_t nfull = (end - begin) / nt;   // iterations in which every lane has a particle
    int64_t i = begin + tid;
    if (nfull >= 2) {
        Regs r = load_particle<MODE, S>(P, cur, i);
        for (int64_t it = 0; it + 1 < nfull; ++it) {
            const Regs rn = load_particle<MODE, S>(P, cur, i + nt);
            process_particle<MODE, S, true>(P, L, i, end, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun, nq);
            r = rn;
            i += nt;
        }
        // iteration nfull - 1, whose successor is the ragged tail (possibly empty)
        const Regs rn = load_particle_if<MODE, S>(P, cur, i + nt, end);
        process_particle<MODE, S, true>(P, L, i, end, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun, nq);
        i += nt;
        process_particle<MODE, S, false>(P, L, i, end, rn, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun, nq);
    } else {
        Regs r = load_particle_if<MODE, S>(P, cur, i, end);
        for (int64_t base = begin; base < end; base += nt) {
            const Regs rn = load_particle_if<MODE, S>(P, cur, i + nt, end);
            process_particle<MODE, S, false>(P, L, i, end, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun,
                                             nq);
            r = rn;
            i += nt;
        }
    }
    if (S == 1) {
        flush_run(L, qrun);
        if (sample) flush_run(L, mrun);
    }
    if ((MODE & kComplete) && nq > 0u) drain_queue<MODE, S>(P, L, wq, nq, nq, stepf, cur, ns0, ns1, sample);
}

// Dynamic work distribution (pass_dyn_kernel, chosen by the host for a single discharge
// whose workgroups each start with at least 2 kPassDynMinShare slots).  A static cut into
// equal slot ranges (run_range) left the last workgroup ~20 us behind the mean at 5x10^7
// particles: the cost of a range varies from step to step.  Here each workgroup's waves take
// sub-blocks of kSubIters iterations over 64 consecutive slots from an LDS counter, so a
// wave that runs ahead takes more; and where every workgroup's share of a species is at
// least kPassDynMinShare slots, the slots of the species are cut into blocks of kBlockSlots
// that the workgroups serving it take from a global counter (kRepBlock + S), so the
// workgroups finish together.  The wave holding a block's first sub-block fetches the
// workgroup's block two ahead, once the block one ahead has been published, so the ids of a
// workgroup's blocks increase and its first kNoBlock means the species is done.  Every wait
// is bounded (kErrSchedule).  Smaller discharges and the batched launch keep the static cut
// (pass_kernel): there the per-wave sub-blocks were slower (measured: +4 % on the
// 2x10^6-particle discharge, +13 % on the 64-discharge batch).
constexpr int kSubIters = 4;
constexpr int kSubSlots = 64 * kSubIters;
constexpr int kBlockSubs = 16;
constexpr int kBlockSlots = kSubSlots * kBlockSubs;
static_assert(kPassDynMinShare == 8 * kBlockSlots, "a workgroup takes at least 8 blocks");
constexpr uint32_t kNoBlock = 0xFFFFFFFFu;
constexpr int kSpinLimit = 1 << 20;

// Where a workgroup's slots of a species come from: blocks from gctr (dyn), else its static
// range [b, e).
struct Dist {
    unsigned long long* gctr;
    uint64_t nblk;
    int64_t b, e;
    bool dyn;
};

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The tagged entry of the workgroup's block j, once published.
__device__ __forceinline__ uint64_t ring_wait(const Lds& L, uint32_t j) {
    for (int k = 0; k < kSpinLimit; ++k) {
        const uint64_t v =
            uniform64(__hip_atomic_load(&L.ring[j % kPassRing], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if ((uint32_t)(v >> 32) == j) return v;
        __builtin_amdgcn_s_sleep(1);
    }
    if ((threadIdx.x & 63) == 0) atomicOr(&L.cnt[kCntErr], kErrSchedule);
    return ((uint64_t)j << 32) | kNoBlock;
}

__device__ __forceinline__ void ring_publish(const Lds& L, uint32_t j, uint32_t id) {
    if ((threadIdx.x & 63) == 0)
        __hip_atomic_store(&L.ring[j % kPassRing], ((uint64_t)j << 32) | id, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Start of the workgroup's distribution for a species (thread 0, before a barrier); with
// blocks, blocks 0 and 1 with one global atomic.
__device__ __forceinline__ void ring_start(const Lds& L, const Dist& d) {
    L.sub[0] = 0u;
    if (!d.dyn) return;
    const uint64_t b = atomicAdd(d.gctr, 2ull);
    for (uint32_t k = 2; k < (uint32_t)kPassRing; ++k) L.ring[k] = ~0ull;   // tags no j reaches
    L.ring[0] = b < d.nblk ? b : (uint64_t)kNoBlock;
    L.ring[1] = (1ull << 32) | (b + 1 < d.nblk ? b + 1 : (uint64_t)kNoBlock);
}

// First slot of this wave's next sub-block, or -1 when the workgroup's part of the species
// (slots below ns) is done (wave-uniform).
__device__ __forceinline__ int64_t next_sub(const Lds& L, const Dist& d, int64_t ns) {
    uint32_t s = 0;
    if ((threadIdx.x & 63) == 0) s = atomicAdd(L.sub, 1u);
    s = __builtin_amdgcn_readfirstlane(s);
    if (!d.dyn) {
        const int64_t base = d.b + (int64_t)s * kSubSlots;
        return base < d.e ? base : -1;
    }
    unsigned long long* gctr = d.gctr;
    const uint64_t nblk = d.nblk;
    const uint32_t j = s / kBlockSubs, q = s % kBlockSubs;
    if (q == 0) {
        uint32_t id = kNoBlock;
        if ((uint32_t)ring_wait(L, j + 1) != kNoBlock) {
            uint64_t b = 0;
            if ((threadIdx.x & 63) == 0) b = atomicAdd(gctr, 1ull);
            b = uniform64(b);
            if (b < nblk) id = (uint32_t)b;
        }
        ring_publish(L, j + 2, id);
    }
    const uint32_t id = (uint32_t)ring_wait(L, j);
    if (id == kNoBlock) return -1;
    const int64_t base = (int64_t)id * kBlockSlots + (int64_t)q * kSubSlots;
    return base < ns ? base : -1;
}

// The slots of species S, one particle per lane per iteration, in sub-blocks taken as
// above, with the next iteration's loads issued before the current particle is processed
// (also across sub-blocks; one copy of the particle code per species keeps the kernel
// within the instruction cache).  While the current and the next sub-block are whole, loads
// and stores are unconditional, so the wait for the current particle's data does not also
// wait for the next one's loads.
template <int MODE, int S>
__device__ __forceinline__ void run_blocks(const Params& P, const Lds& L, const Dist& d, uint32_t stepf, unsigned cur,
                                           int64_t ns0, int64_t ns1, bool sample) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wq = (tid >> 6) * kWaveQueue;
    const int64_t ns = d.dyn ? (S ? ns1 : ns0) : d.e;   // slots below ns are this workgroup's to take
    ChargeRun qrun;
    MomentRun mrun;
    unsigned nq = 0;   // entries in this wave's queue (wave-uniform)
    int64_t base = next_sub(L, d, ns);
    if (base >= 0) {
        int k = 0;   // iteration within the sub-block
        int64_t i = base + lane;
        Regs r = load_particle_if<MODE, S>(P, cur, i, ns);
        for (;;) {
            int64_t nb = base;
            int nk = k + 1;
            if (nk == kSubIters) {
                nb = next_sub(L, d, ns);
                nk = 0;
            }
            if (nb < 0) break;
            const int64_t in = nb + (int64_t)nk * 64 + lane;
            if (base + kSubSlots <= ns && nb + kSubSlots <= ns) {
                const Regs rn = load_particle<MODE, S>(P, cur, in);
                process_particle<MODE, S, true>(P, L, i, ns, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun,
                                                nq);
                r = rn;
            } else {
                const Regs rn = load_particle_if<MODE, S>(P, cur, in, ns);
                process_particle<MODE, S, false>(P, L, i, ns, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun,
                                                 mrun, nq);
                r = rn;
            }
            base = nb;
            k = nk;
            i = in;
        }
        // the wave's last iteration, with nothing to load after it
        process_particle<MODE, S, false>(P, L, i, ns, r, stepf, cur, ns0, ns1, sample, lane, wq, qrun, mrun, nq);
    }
    if (S == 1) {
        flush_run(L, qrun);
        if (sample) flush_run(L, mrun);
    }
    if ((MODE & kComplete) && nq > 0u) drain_queue<MODE, S>(P, L, wq, nq, nq, stepf, cur, ns0, ns1, sample);
}

// ----------------------------------------------------------------------------------
// Poisson solve (one workgroup).
// ----------------------------------------------------------------------------------
// Running sums of a chunk of a_i: n elements, s1 = sum a_i, s2 = sum of the inclusive
// prefix sums of a_i over the chunk.  Chunk A followed by chunk B combine to
// (nA + nB, s1A + s1B, s2A + s2B + nB s1A).
struct Sums2 {
    double n, s1, s2;
};

__device__ __forceinline__ Sums2 combine(const Sums2& a, const Sums2& b) {
    return {a.n + b.n, a.s1 + b.s1, a.s2 + b.s2 + b.n * a.s1};
}

__device__ __forceinline__ Sums2 shfl_up(const Sums2& v, int off) {
    return {__shfl_up(v.n, off, 64), __shfl_up(v.s1, off, 64), __shfl_up(v.s2, off, 64)};
}

// Poisson with phi_0 = phi0, phi_N = 0 (Sec. 2, 2.2; central differences, Sec. 2.3), on
// node charges Qd [C/m^2] in LDS.  With D_i = phi_{i+1} - phi_i the difference equations
// read D_i = D_0 - (dx/eps0) S1_i, S1_i = sum_{k=1..i} Q_k, so
// phi_i = phi0 + i D_0 - (dx/eps0) S2_i with S2_i = sum_{k<i} S1_k, and phi_N = 0 fixes
// D_0 = ((dx/eps0) S2_N - phi0) / N.  One workgroup scan of (n, S1, S2) gives both sums.
// Boundary fields by Gauss's law over the half cells next to the electrodes.  Writes phi
// (FP64, also to phis in LDS) and E (FP32) to global memory; returns E_0 and E_N.
__device__ void solve_field(const Params& P, const double* Qd, double* phis, double* scratch, double phi0,
                            double& E0, double& EN) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    const int nc = P.n_cells, nn = nc + 1;
    const double dxe = P.dx_d / P.eps0;
    // a_i = Q_i for 1 <= i < nc, a_0 = 0; thread tid owns a contiguous chunk
    const int per = (nc + nt - 1) / nt;
    const int b = min(tid * per, nc), e = min(b + per, nc);
    Sums2 loc{(double)(e - b), 0.0, 0.0};
    for (int i = b; i < e; ++i) {
        loc.s1 += (i >= 1) ? Qd[i] : 0.0;
        loc.s2 += loc.s1;
    }
    Sums2 inc = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const Sums2 t = shfl_up(inc, off);
        if (lane >= off) inc = combine(t, inc);
    }
    Sums2* wsum = reinterpret_cast<Sums2*>(scratch);   // nw <= 16 entries
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    Sums2 before{0.0, 0.0, 0.0}, total{0.0, 0.0, 0.0};
    for (int w = 0; w < nw; ++w) {
        if (w == wid) before = total;
        total = combine(total, wsum[w]);
    }
    // exclusive prefix of this thread's chunk
    Sums2 ex = shfl_up(inc, 1);
    if (lane == 0) ex = {0.0, 0.0, 0.0};
    ex = combine(before, ex);
    const double D0 = (dxe * total.s2 - phi0) / (double)nc;
    double s1 = ex.s1, s2 = ex.s2;   // S1_{i-1} and S2_i at the chunk start
    for (int i = b; i < e; ++i) {
        const double ph = (i == 0) ? phi0 : phi0 + (double)i * D0 - dxe * s2;
        phis[i] = ph;
        P.phi[i] = ph;
        s1 += (i >= 1) ? Qd[i] : 0.0;
        s2 += s1;
    }
    if (tid == 0) {
        phis[nc] = 0.0;
        P.phi[nc] = 0.0;
    }
    __syncthreads();
    const double inv2dx = 0.5 / P.dx_d, invdx = 1.0 / P.dx_d;
    for (int i = tid; i < nn; i += nt) {
        double ef;
        if (i == 0)
            ef = (phis[0] - phis[1]) * invdx - Qd[0] / P.eps0;
        else if (i == nc)
            ef = (phis[nc - 1] - phis[nc]) * invdx + Qd[nc] / P.eps0;
        else
            ef = (phis[i - 1] - phis[i + 1]) * inv2dx;
        P.E[i] = (float)ef;
        if (i == 0) scratch[48] = ef;
        if (i == nc) scratch[49] = ef;
    }
    __syncthreads();
    E0 = scratch[48];
    EN = scratch[49];
}

// Bitonic sort of keys[0..n2) ascending, n2 a power of two.  Element k is owned by thread
// k % blockDim, in lane k % 64 of its wave; compare-exchange partners closer than 64 are in
// the same wave and are exchanged with cross-lane shuffles in registers, farther ones
// through LDS, so only strides >= 64 need a workgroup barrier.  (For n2 >= 64 every lane
// of a wave owns an element in the same round; below, all partners are owned.)
__device__ __forceinline__ uint32_t bitonic_lanes(uint32_t x, unsigned k, unsigned size_lo, unsigned size_hi,
                                                  unsigned top) {
    for (unsigned sz = size_lo; sz <= size_hi; sz <<= 1)
        for (unsigned st = min(sz >> 1, top); st > 0; st >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)x, (int)st, 64);
            const bool up = (k & sz) == 0;
            const bool lower = (k & st) == 0;
            x = (lower == up) ? min(x, o) : max(x, o);
        }
    return x;
}

__device__ void bitonic_sort(uint32_t* keys, unsigned n2) {
    const unsigned tid = threadIdx.x, nt = blockDim.x;
    if (n2 < 2) return;
    for (unsigned k = tid; k < n2; k += nt) keys[k] = bitonic_lanes(keys[k], k, 2, min(n2, 64u), 32);
    __syncthreads();
    for (unsigned size = 128; size <= n2; size <<= 1) {
        for (unsigned stride = size >> 1; stride >= 64; stride >>= 1) {
            for (unsigned t = tid; t < n2; t += nt) {
                const unsigned partner = t ^ stride;
                if (partner > t) {
                    const bool up = (t & size) == 0;
                    const uint32_t a = keys[t], c = keys[partner];
                    if ((a > c) == up) {
                        keys[t] = c;
                        keys[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
        for (unsigned k = tid; k < n2; k += nt) keys[k] = bitonic_lanes(keys[k], k, size, size, 32);
        __syncthreads();
    }
}

// In-place inclusive prefix sum of v[0..n) by one workgroup (blockDim a multiple of 64):
// each thread sums a contiguous run, the run totals are scanned across the wave with
// shuffles and across waves through part[blockDim / 64].
__device__ void block_inclusive_scan(uint32_t* v, unsigned n, uint32_t* part) {
    const unsigned tid = threadIdx.x, nt = blockDim.x, lane = tid & 63u, wv = tid >> 6;
    const unsigned c = (n + nt - 1) / nt, b0 = min(tid * c, n), b1 = min(b0 + c, n);
    uint32_t run = 0;
    for (unsigned i = b0; i < b1; ++i) run += v[i];
    uint32_t x = run;
    for (unsigned d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) part[wv] = x;
    __syncthreads();
    uint32_t acc = x - run;
    for (unsigned w = 0; w < wv; ++w) acc += part[w];
    for (unsigned i = b0; i < b1; ++i) {
        acc += v[i];
        v[i] = acc;
    }
    __syncthreads();
}

// Ids of this launch's ionisation products: the k-th parent in ascending id order gives
// next_id_e + k and next_id_i + k (parents are distinct electrons).  Up to kBirthSortCap
// parents are sorted in LDS and each finds its rank by binary search.  More are binned by
// their leading id bits (a bin index that never decreases with the id): bin starts come
// from a prefix sum of the bin counts, the parents are scattered to bin order in
// P.birth_order, and a parent's rank is its bin's start plus the smaller ids in its bin,
// so the work grows with the births times the mean bin occupancy.  keys and parents are
// kBirthSortCap words each, contiguous; part holds blockDim / 64 words.
__device__ void assign_birth_ids(const Params& P, uint32_t* keys, uint32_t* parents, uint32_t* part, unsigned cur,
                                 int64_t ns0, int64_t ns1, unsigned nbv, int64_t nid0, int64_t nid1) {
    const int tid = threadIdx.x, nt = blockDim.x;
    if (nbv == 0) return;
    if (nbv <= (unsigned)kBirthSortCap) {
        unsigned n2 = 1;
        while (n2 < nbv) n2 <<= 1;
        for (unsigned k = tid; k < n2; k += nt) {
            const uint32_t p = k < nbv ? ld_agent(&P.birth_parent[k]) : 0xFFFFFFFFu;
            keys[k] = p;
            parents[k] = p;
        }
        __syncthreads();
        bitonic_sort(keys, n2);
        for (unsigned k = tid; k < nbv; k += nt) {
            const uint32_t p = parents[k];
            unsigned lo = 0, hi = nbv;
            while (lo < hi) {
                const unsigned mid = (lo + hi) >> 1;
                if (keys[mid] < p) lo = mid + 1; else hi = mid;
            }
            bufsel(P.id, cur, 0)[ns0 + k] = (uint32_t)(nid0 + lo);
            bufsel(P.id, cur, 1)[ns1 + k] = (uint32_t)(nid1 + lo);
        }
        __syncthreads();
        return;
    }
    // bins 0..kBins-1 plus an end entry fill keys and parents
    constexpr unsigned kBins = 2u * (unsigned)kBirthSortCap - 1u;
    uint32_t* bin = keys;
    // parent ids are below nid0 <= 2^32: keep their leading 12 bits
    const unsigned bits = nid0 > 1 ? 64u - (unsigned)__clzll((unsigned long long)(nid0 - 1)) : 1u;
    const unsigned sh = bits > 12u ? bits - 12u : 0u;
    for (unsigned b = tid; b <= kBins; b += nt) bin[b] = 0u;
    __syncthreads();
    for (unsigned k = tid; k < nbv; k += nt) atomicAdd(&bin[min(ld_agent(&P.birth_parent[k]) >> sh, kBins - 1u)], 1u);
    __syncthreads();
    block_inclusive_scan(bin, kBins, part);   // bin[b] = end of bin b
    if (tid == 0) bin[kBins] = nbv;
    for (unsigned k = tid; k < nbv; k += nt) {
        const uint32_t p = ld_agent(&P.birth_parent[k]);
        const unsigned pos = atomicSub(&bin[min(p >> sh, kBins - 1u)], 1u) - 1u;
        st_agent(&P.birth_order[pos], ((unsigned long long)p << 32) | k);
    }
    // now bin[b] = start of bin b and bin[b + 1] its end; the scattered entries are read
    // back by other waves of this workgroup
    __threadfence();
    __syncthreads();
    for (unsigned j = tid; j < nbv; j += nt) {
        const unsigned long long e = ld_agent(&P.birth_order[j]);
        const uint32_t p = (uint32_t)(e >> 32), k = (uint32_t)e;
        const unsigned b = min(p >> sh, kBins - 1u), hi = bin[b + 1];
        unsigned rank = bin[b];
        for (unsigned q = bin[b]; q < hi; ++q) rank += (uint32_t)(ld_agent(&P.birth_order[q]) >> 32) < p;
        bufsel(P.id, cur, 0)[ns0 + k] = (uint32_t)(nid0 + rank);
        bufsel(P.id, cur, 1)[ns1 + k] = (uint32_t)(nid1 + rank);
    }
    __syncthreads();
}

// LDS layout of the epilogue (bytes): control block copy, then FP64 node arrays.
constexpr int kEpiCtrlBytes = 512;
static_assert(sizeof(Ctrl) <= kEpiCtrlBytes && sizeof(Ctrl) % 8 == 0, "control block copy");
constexpr int kEpiNodesPerThread = 8;   // the host keeps n_cells + 1 <= 8 * blockDim

// Work of the last workgroup of a launch.  The control block and the charge grid are
// loaded in one round trip, the bookkeeping and the Poisson solve run in LDS, and all
// results are stored at the end.  When the step just started will be sampled, the window
// sums receive its densities (the deposit of its positions) and its potential here; its
// completion adds the rest of the sample.
template <int MODE>
__device__ void epilogue(const Params& P, unsigned char* smem, int64_t step, unsigned cur, int64_t ns0,
                         int64_t ns1, bool sample) {
    Ctrl* C = P.ctrl;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nc = P.n_cells, nn = nc + 1;
    Ctrl* cs = reinterpret_cast<Ctrl*>(smem);
    double* Qd = reinterpret_cast<double*>(smem + kEpiCtrlBytes);
    double* dep0 = Qd + nn;      // this launch's deposit per species [particles]
    double* dep1 = dep0 + nn;
    double* scratch = dep1 + nn;                                  // 64 doubles
    // the birth ranking is done before the solve needs phis
    double* phis = scratch + 64;
    uint32_t* keys = reinterpret_cast<uint32_t*>(phis);           // kBirthSortCap
    uint32_t* parents = keys + kBirthSortCap;                     // kBirthSortCap
    constexpr bool kSolve = (MODE & (kAdvance | kDeposit)) != 0;
    constexpr int kWords = (int)(sizeof(Ctrl) / 8);
    __syncthreads();   // the particle pass is done with LDS

    // ---- one round trip of loads
    unsigned long long* cw = reinterpret_cast<unsigned long long*>(cs);
    unsigned long long* gw = reinterpret_cast<unsigned long long*>(C);
    for (int w = tid; w < kWords; w += nt) cw[w] = ld_agent(&gw[w]);
    if (kSolve) {
        unsigned long long q0[kEpiNodesPerThread], q1[kEpiNodesPerThread];
#pragma unroll
        for (int r = 0; r < kEpiNodesPerThread; ++r) {
            const int i = tid + r * nt;
            q0[r] = i < nn ? __hip_atomic_exchange(&P.Qs[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
            q1[r] = i < nn ? __hip_atomic_exchange(&P.Qs[nn + i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : 0ull;
        }
        const double scale = kQScaleInv * P.e0W;
#pragma unroll
        for (int r = 0; r < kEpiNodesPerThread; ++r) {
            const int i = tid + r * nt;
            if (i < nn) {
                Qd[i] = (double)((long long)q1[r] - (long long)q0[r]) * scale;
                dep0[i] = (double)q0[r] * kQScaleInv;
                dep1[i] = (double)q1[r] * kQScaleInv;
            }
        }
    }
    __syncthreads();

    // ---- the workgroups' counters, summed over the sets (which are cleared for the next launch)
    if (tid < kRepDone) {
        unsigned long long v = 0;
        for (int q = 0; q < kRepSets; ++q) {
            const unsigned long long x = ld_agent(&P.rep[q * kRepStride + tid]);
            v = (tid == kRepErr) ? (v | x) : (v + x);
        }
        if (tid < kRepColl) cs->absorbed_step[(tid - kRepAbs) >> 1][(tid - kRepAbs) & 1] += v;
        else if (tid < kRepViol) cs->coll[tid - kRepColl] += v;
        else if (tid < kRepErr) cs->viol[tid - kRepViol] += v;
        else if (tid == kRepErr) atomicOr(&cs->err, (unsigned)v);
        else if (tid < kRepParts) cs->cost_ticks[tid - kRepTicks] = v;
        else cs->cost_parts[tid - kRepParts] = v;
    }
    __syncthreads();
    for (int w = tid; w < kRepSets * kRepStride; w += nt) P.rep[w] = 0ull;
    // ---- completion of the previous step: births
    if (MODE & kComplete) {
        const unsigned nb = cs->n_births;
        unsigned nbv = nb;
        if ((int64_t)nbv > P.max_births) nbv = (unsigned)P.max_births;
        if ((int64_t)nbv > P.cap[0] - ns0) nbv = (unsigned)(P.cap[0] - ns0);
        if ((int64_t)nbv > P.cap[1] - ns1) nbv = (unsigned)(P.cap[1] - ns1);
        const int64_t nid0 = cs->next_id[0], nid1 = cs->next_id[1];
        assign_birth_ids(P, keys, parents, reinterpret_cast<uint32_t*>(scratch), cur, ns0, ns1, nbv, nid0, nid1);
        if (tid == 0) {
            if (nb > nbv) cs->err |= (nbv == (unsigned)P.max_births) ? kErrBirths : kErrCapacity;
            if (nid0 + nbv > 0x100000000ll || nid1 + nbv > 0x100000000ll) cs->err |= kErrIds;
            cs->n_slots[0] = ns0 + nbv;
            cs->n_slots[1] = ns1 + nbv;
            cs->next_id[0] = nid0 + nbv;
            cs->next_id[1] = nid1 + nbv;
            cs->n_alive[0] += nbv;
            cs->n_alive[1] += nbv;
            cs->births_total += nbv;
            cs->births_lost += nb - nbv;
            cs->n_births = 0;
            if (sample) cs->n_samples += 1;
        }
        __syncthreads();
    }

    // ---- the field for the new time level
    if (kSolve) {
        double E0, EN;
        const double t1 = (double)(step + ((MODE & kAdvance) ? 1 : 0)) * P.dt_d;
        solve_field(P, Qd, phis, scratch, cs->V0 * sin(P.omega * t1), E0, EN);
        // the step just started is sampled at its completion: densities at x^{n+1} are
        // this launch's deposit, and phi^{n+1} was just solved for
        const bool next_sampled = (MODE & kAdvance) && ((step + 1) % P.moments_every == 0);
        for (int i = tid; i < nn; i += nt) {
            P.Q_last[i] = Qd[i];
            if (next_sampled) {
                unsafeAtomicAdd(&P.mom[i], dep0[i]);
                unsafeAtomicAdd(&P.mom[nn + i], dep1[i]);
                unsafeAtomicAdd(&P.mom[4 * nn + i], phis[i]);
            }
        }
        if (tid == 0) {
            if (MODE & kAdvance) {
                unsigned long long a[2][2];
                for (int s = 0; s < 2; ++s)
                    for (int e = 0; e < 2; ++e) {
                        a[s][e] = cs->absorbed_step[s][e];
                        cs->absorbed_step[s][e] = 0;
                        cs->absorbed_total[s][e] += a[s][e];
                        cs->absorbed_window[s][e] += a[s][e];
                    }
                cs->particle_steps += cs->n_alive[0] + cs->n_alive[1];
                cs->n_alive[0] -= (int64_t)(a[0][0] + a[0][1]);
                cs->n_alive[1] -= (int64_t)(a[1][0] + a[1][1]);
                const double J = P.eps0 * (E0 - cs->E0_prev) / P.dt_d +
                                 P.e0W * ((double)a[0][0] - (double)a[1][0]) / P.dt_d;
                cs->J_last = J;
                const int64_t n1 = step + 1;
                if (P.flux_trace) {   // fluxes at the powered electrode against time
                    unsigned long long* ft = P.flux_trace + 2 * ((n1 - 1) % P.steps_per_period);
                    ft[0] = a[0][0];
                    ft[1] = a[1][0];
                }
                cs->J_period_max = fmax(cs->J_period_max, fabs(J));
                if (n1 % P.steps_per_period == 0) {
                    if (cs->period_valid) {
                        cs->J_max_sum += cs->J_period_max;
                        cs->n_periods += 1;
                        // current-driven operation (Sec. 2, Eq. "adaptivevoltage"): the next
                        // period runs at V0 J0 / J_calc, J_calc this period's max |J|
                        if (P.J0_target > 0.0 && cs->J_period_max > 0.0)
                            cs->V0 *= P.J0_target / cs->J_period_max;
                    }
                    cs->J_period_max = 0.0;
                    cs->period_valid = 1;
                }
                cs->n_steps_window += 1;
                cs->step = n1;
            }
            cs->E0_prev = E0;
            cs->sigma0 = P.eps0 * E0;
            cs->sigmad = -P.eps0 * EN;
        }
    }
    if (tid == 0) {
        cs->done = 0;
        if ((MODE & kAdvance) && cs->cost_parts[0] > 0 && cs->cost_parts[1] > 0 && cs->cost_ticks[1] > 0) {
            const double r = ((double)cs->cost_ticks[0] / (double)cs->cost_parts[0]) /
                             ((double)cs->cost_ticks[1] / (double)cs->cost_parts[1]);
            cs->cost_ratio = fmin(4.0, fmax(0.25, 0.95 * cs->cost_ratio + 0.05 * r));
        }
        for (int q = 0; q < 2; ++q) {
            cs->cost_ticks[q] = 0;
            cs->cost_parts[q] = 0;
        }
    }
    __syncthreads();
    for (int w = tid; w < kWords; w += nt) gw[w] = cw[w];
}

// One launch's work of workgroup wg of the G workgroups that serve discharge P.
template <int MODE, bool DYN>
__device__ __forceinline__ void pass_body(const Params& P, unsigned char* smem, const int wg, const int G) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nn = P.n_cells + 1;
    Ctrl* C = P.ctrl;
    Lds L;
    L.cnt = reinterpret_cast<uint32_t*>(smem);
    L.ring = reinterpret_cast<unsigned long long*>(smem + kCntSlots * 4);
    L.sub = reinterpret_cast<uint32_t*>(L.ring + kPassRing);
    L.Q = reinterpret_cast<unsigned long long*>(smem + kCntSlots * 4 + kPassRingBytes);
    L.M = L.Q + nn;
    L.E = reinterpret_cast<float*>(L.M + nn);
    L.U = L.E + nn;
    const int qcap = (nt >> 6) * kWaveQueue;
    L.qslot = reinterpret_cast<uint32_t*>(L.U + kNullBins + 1);
    L.qr = L.qslot + qcap;
    L.qvx = reinterpret_cast<float*>(L.qr + qcap);
    L.qx = L.qvx + qcap;
    L.qid = reinterpret_cast<uint32_t*>(L.qx + qcap);
    L.qvy = reinterpret_cast<float*>(L.qid + qcap);
    L.qvz = L.qvy + qcap;

    const int64_t step = C->step;
    const unsigned cur = C->cur;
    const int64_t ns0 = C->n_slots[0], ns1 = C->n_slots[1];
    const bool sample = (MODE & kComplete) && (step % P.moments_every == 0);
    const uint32_t stepf = (uint32_t)step;

    for (int i = tid; i < kCntSlots; i += nt) L.cnt[i] = 0;
    if (MODE != kDeposit)
        for (int i = tid; i < nn; i += nt) L.E[i] = P.E[i];
    if (MODE & kComplete)
        for (int i = tid; i <= kNullBins; i += nt) L.U[i] = P.nullbound[i];

    // Workgroups are species-pure: the first G_e serve the electrons, the rest the ions, G_e in
    // proportion to the expected work, slot counts weighted by the measured cost per slot of
    // each species (a single workgroup serves both, one after the other).  Within a species
    // the slots go to waves in sub-blocks as they ask for them (run_blocks).
    int64_t b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    bool dyn0 = false, dyn1 = false;   // blocks from the global counter (DYN only)
    if (G == 1) {
        e0 = ns0;
        e1 = ns1;
    } else {
        const double w0 = (double)ns0 * C->cost_ratio, w1 = (double)ns1;
        int Ge = (w0 + w1) > 0.0 ? (int)((double)G * w0 / (w0 + w1) + 0.5) : G / 2;
        if (ns0 > 0) Ge = max(Ge, 1);
        if (ns1 > 0) Ge = min(Ge, G - 1);
        if (ns1 == 0) Ge = G;
        const int b = wg;
        if (b < Ge) {
            const int64_t per = (ns0 + Ge - 1) / Ge;
            b0 = min((int64_t)b * per, ns0);
            e0 = min(b0 + per, ns0);
            dyn0 = DYN && Ge > 1 && per >= kPassDynMinShare;
        } else {
            const int Gi = G - Ge;
            const int64_t per = (ns1 + Gi - 1) / Gi;
            b1 = min((int64_t)(b - Ge) * per, ns1);
            e1 = min(b1 + per, ns1);
            dyn1 = DYN && Gi > 1 && per >= kPassDynMinShare;
        }
    }
    for (int s = 0; s < 2; ++s) {
        const int64_t b = s ? b1 : b0, e = s ? e1 : e0;
        if (!(e > b)) continue;
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        for (int i = tid; i < nn; i += nt) {
            L.Q[i] = 0ull;
            if (sample) L.M[i] = 0ull;
        }
        const Dist d{P.rep + kRepBlock + s, (uint64_t)(((s ? ns1 : ns0) + kBlockSlots - 1) / kBlockSlots), b, e,
                     s ? dyn1 : dyn0};
        if (DYN && tid == 0) ring_start(L, d);
        __syncthreads();
        if (DYN) {
            if (s == 0)
                run_blocks<MODE, 0>(P, L, d, stepf, cur, ns0, ns1, sample);
            else
                run_blocks<MODE, 1>(P, L, d, stepf, cur, ns0, ns1, sample);
        } else {
            if (s == 0)
                run_range<MODE, 0>(P, L, b, e, stepf, cur, ns0, ns1, sample);
            else
                run_range<MODE, 1>(P, L, b, e, stepf, cur, ns0, ns1, sample);
        }
        __syncthreads();
        if (tid == 0 && (MODE & kAdvance)) {   // balance data for the next launch's split
            L.cnt[kCntTicks + s] = (uint32_t)(__builtin_amdgcn_s_memrealtime() - t0);
            L.cnt[kCntParts + s] = (uint32_t)(e - b);
        }
        // this species' deposit, and its energy (e) or v_x (i) sums
        unsigned long long* qg = P.Qs + s * nn;
        double* sec = P.mom + (s ? 3 * nn : 2 * nn);
        const double inv2 = 1.0 / P.mscale[s];
        for (int i = tid; i < nn; i += nt) {
            const unsigned long long q = L.Q[i];
            if (q != 0ull) atomicAdd(&qg[i], q);
            if (sample) {
                const long long m1 = (long long)L.M[i];
                if (m1 != 0) unsafeAtomicAdd(&sec[i], (double)m1 * inv2);
            }
        }
        __syncthreads();
    }
    // this workgroup's counters to its set (LDS slot k maps to set word k, see kRep*)
    const int set = wg % kRepSets;
    unsigned long long* rs = P.rep + set * kRepStride;
    if (tid < kCntErr) {
        if (L.cnt[tid]) atomicAdd(&rs[tid], (unsigned long long)L.cnt[tid]);
    } else if (tid == kCntErr) {
        if (L.cnt[tid]) atomicOr(&rs[kRepErr], (unsigned long long)L.cnt[tid]);
    } else if (tid < kCntErr + 5) {   // ticks and slots of the species run
        if (L.cnt[tid]) atomicAdd(&rs[tid], (unsigned long long)L.cnt[tid]);
    }
    wait_memory_complete();
    __syncthreads();
    if (tid == 0) {
        // two-level completion count: the last workgroup of its set counts the set
        const unsigned members = (unsigned)((G - set + kRepSets - 1) / kRepSets);
        const unsigned sets = (unsigned)min(G, kRepSets);
        unsigned last = 0;
        if (atomicAdd(&rs[kRepDone], 1ull) == members - 1) last = atomicAdd(&C->done, 1u) == sets - 1 ? 1u : 0u;
        L.cnt[kCntLast] = last;
    }
    __syncthreads();
    if (!L.cnt[kCntLast]) return;
    epilogue<MODE>(P, smem, step, cur, ns0, ns1, sample);
}

template <int MODE>
__global__ void __launch_bounds__(1024) pass_kernel(Params P) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass_body<MODE, false>(P, smem, blockIdx.x, gridDim.x);
}

// The same launch with the dynamic work distribution (run_blocks).
template <int MODE>
__global__ void __launch_bounds__(1024) pass_dyn_kernel(Params P) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass_body<MODE, true>(P, smem, blockIdx.x, gridDim.x);
}

// Several independent discharges advanced by one launch: discharge d owns workgroups
// [seg[d], seg[d+1]) and its parameters are batch[d]; each discharge's last workgroup runs
// its own epilogue.  Every discharge takes the same step mode.
template <int MODE>
__global__ void __launch_bounds__(1024) pass_batch_kernel(const Params* __restrict__ batch,
                                                          const int* __restrict__ seg, int nd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    int lo = 0, hi = nd;   // seg[lo] <= b < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= b) lo = mid; else hi = mid;
    }
    pass_body<MODE, false>(batch[lo], smem, b - seg[lo], seg[lo + 1] - seg[lo]);
}

// ----------------------------------------------------------------------------------
// Initial load (Sec. 2.2): uniform positions, Maxwellian velocities, ids 0..n-1.
// ----------------------------------------------------------------------------------
__global__ void load_kernel(Params P, int s, int64_t n, double vth) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t tag = ((uint32_t)s << 8) | kLoad;
    const uint4 A = philox((uint32_t)k, 0u, 0u, tag, P.key0, P.key1);
    const uint4 B = philox((uint32_t)k, 0u, 1u, tag, P.key0, P.key1);
    // x = d u in metres, i.e. n_cells u in cell units
    float x = (float)((double)P.n_cells * u01d(A.x));
    if (!(x < P.ncf)) x = nextafterf(P.ncf, 0.0f);
    const double r0 = sqrt(-2.0 * log(u01d(A.y)));
    double s0, c0, s1, c1;
    sincospi(2.0 * u01d(A.z), &s0, &c0);
    const double r1 = sqrt(-2.0 * log(u01d(B.x)));
    sincospi(2.0 * u01d(B.y), &s1, &c1);
    P.x[0][s][k] = x;
    P.vx[0][s][k] = (float)(vth * r0 * c0);
    P.vy[0][s][k] = (float)(vth * r0 * s0);
    P.vz[0][s][k] = (float)(vth * r1 * c1);
    P.id[0][s][k] = (uint32_t)k;
}

// Warm-start load of species s from profiles on np equally spaced points spanning the gap
// (linear in between): tab = [C | n | v2 | u], np entries each, with C the cumulative
// integral of the density n (trapezoids of width h_m metres), v2 the thermal speed squared
// per component and u the mean v_x.  Particle k inverts C at u01 * C[np - 1] (segment by
// binary search, then the root of a t + (b - a) t^2 / 2 = (c - C_j) / h_m), takes a
// Maxwellian velocity with v2 and u interpolated at its position, and id k.  Counters
// (k, 0, 0 and 1, (s << 8) | kWarm).
__global__ void load_profile_kernel(Params P, int s, int64_t n, unsigned b, const double* __restrict__ tab, int np,
                                    double h_m) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t tag = ((uint32_t)s << 8) | kWarm;
    const uint4 A = philox((uint32_t)k, 0u, 0u, tag, P.key0, P.key1);
    const uint4 B = philox((uint32_t)k, 0u, 1u, tag, P.key0, P.key1);
    const double* C = tab;
    const double* dens = tab + np;
    const double* v2 = tab + 2 * np;
    const double* drift = tab + 3 * np;
    const double c = u01d(A.x) * C[np - 1];
    int lo = 0, hi = np - 1;   // the last j <= np - 2 with C[j] <= c
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (C[mid] <= c) lo = mid; else hi = mid;
    }
    const int j = lo;
    const double a = dens[j], bb = dens[j + 1];
    const double q = (c - C[j]) / h_m;
    const double disc = sqrt(fmax(a * a + 2.0 * (bb - a) * q, 0.0));
    double t = (a + disc > 0.0) ? 2.0 * q / (a + disc) : 0.5;
    t = fmin(fmax(t, 0.0), 1.0);
    float x = (float)(((double)j + t) * ((double)P.n_cells / (double)(np - 1)));
    if (!(x < P.ncf)) x = nextafterf(P.ncf, 0.0f);
    if (!(x > 0.0f)) x = 1.0e-30f;
    const double vth = sqrt((1.0 - t) * v2[j] + t * v2[j + 1]);
    const double um = (1.0 - t) * drift[j] + t * drift[j + 1];
    const double r0 = sqrt(-2.0 * log(u01d(A.y)));
    double s0, c0, s1, c1;
    sincospi(2.0 * u01d(A.z), &s0, &c0);
    const double r1 = sqrt(-2.0 * log(u01d(B.x)));
    sincospi(2.0 * u01d(B.y), &s1, &c1);
    P.x[b][s][k] = x;
    P.vx[b][s][k] = (float)(vth * r0 * c0 + um);
    P.vy[b][s][k] = (float)(vth * r0 * s0);
    P.vz[b][s][k] = (float)(vth * r1 * c1);
    P.id[b][s][k] = (uint32_t)k;
}

// ----------------------------------------------------------------------------------
// Diagnostics of one sample of the completed state (the paper's results section: EEDF,
// fast electrons, heating, ionisation rate, particle and energy fluxes).  They run between
// steps, on demand, and leave the particle pass untouched.
// ----------------------------------------------------------------------------------
// n_gas sigma [1/m] of process p at frame energy eps [eV], by the particle pass's rule:
// zero below the threshold, the energy raised to the floor, the last point at or beyond the
// table end, linear interpolation in between.
__device__ __forceinline__ float table_ngs(const Params& P, const ProcDev& p, float eps) {
    if (eps < p.thr) return 0.0f;
    const float t = fmaxf(eps, p.emin) * p.inv_de;
    const bool top = t >= (float)(p.n - 1);
    const int kk = top ? p.n - 2 : (int)t;
    const float a = P.tab[p.off + kk], b = P.tab[p.off + kk + 1];
    return top ? b : fmaf(b - a, t - (float)kk, a);
}

// Each workgroup sums its electrons in LDS (six node grids: weight, U, e0 U v_x, expected
// ionisation rate n_gas sigma_iz(U) |v|, fast (U > |V0| / 4 with the amplitude in use), v_x;
// and the energy histogram), then adds them to the window (v_x to this sample's grid).
__global__ void __launch_bounds__(256) diag_kernel(Params P, DiagDev D) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nn = P.n_cells + 1, tid = threadIdx.x, nt = blockDim.x;
    float* acc = reinterpret_cast<float*>(smem);
    unsigned* hist = reinterpret_cast<unsigned*>(acc + 6 * nn);
    __shared__ unsigned wcount;
    for (int i = tid; i < 6 * nn; i += nt) acc[i] = 0.0f;
    for (int i = tid; i < D.n_bins; i += nt) hist[i] = 0u;
    if (tid == 0) wcount = 0u;
    __syncthreads();
    const Ctrl* C = P.ctrl;
    const unsigned cur = C->cur;
    const int64_t ns = C->n_slots[0];
    const float fast = 0.25f * (float)fabs(C->V0);
    const float* X = bufsel(P.x, cur, 0);
    const float* VX = bufsel(P.vx, cur, 0);
    const float* VY = bufsel(P.vy, cur, 0);
    const float* VZ = bufsel(P.vz, cur, 0);
    unsigned cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * nt + tid; i < ns; i += (int64_t)gridDim.x * nt) {
        const float x = X[i];
        if (!(x > 0.0f)) continue;
        const float vx = VX[i], vy = VY[i], vz = VZ[i];
        const float g2 = vx * vx + vy * vy + vz * vz;
        const float U = P.half_m_over_e[0] * g2;
        const float g = sqrtf(g2);
        float nu = 0.0f;
        for (int k = 0; k < D.n_iz; ++k) {
            const ProcDev& p = P.proc[0][D.iz[k]];
            nu += table_ngs(P, p, p.efac * g2) * g;
        }
        int j;
        float w;
        cell_of(x, P.n_cells, j, w);
        const float vals[6] = {1.0f, U, (float)D.e0 * U * vx, nu, U > fast ? 1.0f : 0.0f, vx};
        for (int q = 0; q < 6; ++q) {
            atomicAdd(&acc[q * nn + j], (1.0f - w) * vals[q]);
            atomicAdd(&acc[q * nn + j + 1], w * vals[q]);
        }
        const float b = U * D.bins_per_eV;
        if (b < (float)D.n_bins) atomicAdd(&hist[(int)b], 1u);
        ++cnt;
    }
    if (cnt) atomicAdd(&wcount, cnt);
    __syncthreads();
    for (int i = tid; i < 6 * nn; i += nt) {
        const float v = acc[i];
        if (v == 0.0f) continue;
        const int q = i / nn, node = i - q * nn;
        if (q == 5) unsafeAtomicAdd(&D.fx_sample[node], (double)v);
        else unsafeAtomicAdd(&D.node[q * nn + node], (double)v);
    }
    for (int i = tid; i < D.n_bins; i += nt)
        if (hist[i]) atomicAdd(&D.hist[i], (unsigned long long)hist[i]);
    if (tid == 0 && wcount) atomicAdd(&D.counts[0], (unsigned long long)wcount);
}

// The sample's node terms: v_x sums into the window, heating -e0 E_i (sum v_x)_i and the
// field E_i of this time level; clears the sample grid and counts the sample.
__global__ void diag_nodes_kernel(Params P, DiagDev D) {
    const int nn = P.n_cells + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x) {
        const double fx = D.fx_sample[i];
        const double E = (double)P.E[i];
        D.node[5 * nn + i] += fx;
        D.node[6 * nn + i] += -D.e0 * E * fx;
        D.node[7 * nn + i] += E;
        D.fx_sample[i] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) D.counts[1] += 1ull;
}

// ----------------------------------------------------------------------------------
// Periodic reordering (performance only; results do not depend on the order because
// every random number is keyed by particle id and the deposits are exact).  A species is
// either sorted by cell (ions, which move a small fraction of a cell per step, keeping the
// per-lane run caches of the particle pass effective; electrons when they stay near
// their cell over a sort interval) or only compacted: absorbed slots removed, order kept,
// which streams.  Counters: cnt[s nc + j] count of cell j of species s (cell sort),
// cnt[2 nc + b] alive particles of block b (compaction); cursor[] holds the matching
// exclusive prefix sums.
// ----------------------------------------------------------------------------------
// Adds this wave's particles to the per-cell counts h (cell j, or -1 for a hole or an
// inactive lane) with one LDS atomic per distinct cell instead of one per particle: a
// cell-sorted wave holds one or two cells, and same-address atomics from the lanes of a
// wave would be serialised.  Returns, per lane, the count of its cell before this wave's
// first lane of that cell plus its rank among the wave's lanes of the cell (unused when
// want_pos is false).  Every lane of the wave must call this.
__device__ __forceinline__ unsigned wave_cell_add(unsigned* h, int j, bool want_pos) {
    const int lane = threadIdx.x & 63;
    unsigned long long todo = __ballot(j >= 0);
    unsigned pos = 0;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int jl = __shfl(j, leader, 64);
        const unsigned long long same = __ballot(j == jl) & todo;
        unsigned base = 0;
        if (lane == leader) {
            const unsigned got = atomicAdd(&h[jl], (unsigned)__popcll(same));
            base = want_pos ? got : 0u;
        }
        base = (unsigned)__shfl((int)base, leader, 64);
        if (j == jl) pos = base + (unsigned)__popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
    return pos;
}

constexpr int kSortUnroll = 4;   // elements per thread per iteration of the reordering loops

// Blocks [0, Ge) take contiguous electron ranges, [Ge, G) ion ranges (G >= 2 when both
// species have slots).
__device__ __forceinline__ void sort_split(int G, int b, int64_t ns0, int64_t ns1, int& s, int& Ge, int64_t& begin,
                                           int64_t& end) {
    const int64_t total = ns0 + ns1;
    Ge = total > 0 ? (int)(((double)G * (double)ns0) / (double)total + 0.5) : G / 2;
    if (ns0 > 0) Ge = max(Ge, 1);
    if (ns1 > 0) Ge = min(Ge, G - 1);
    if (ns1 == 0) Ge = G;
    if (b < Ge) {
        s = 0;
        const int64_t per = (ns0 + Ge - 1) / max(Ge, 1);
        begin = min((int64_t)b * per, ns0);
        end = min(begin + per, ns0);
    } else {
        s = 1;
        const int Gi = G - Ge;
        const int64_t per = (ns1 + Gi - 1) / max(Gi, 1);
        begin = min((int64_t)(b - Ge) * per, ns1);
        end = min(begin + per, ns1);
    }
}

// Block blk of the G blocks that reorder one discharge.
__device__ __forceinline__ void sort_count_body(const Params& P, unsigned* cnt, int G, int blk,
                                                unsigned char* smem) {
    unsigned* h = reinterpret_cast<unsigned*>(smem);   // nc cell counts, then one alive count
    const int nc = P.n_cells, tid = threadIdx.x, nt = blockDim.x;
    const Ctrl* C = P.ctrl;
    const unsigned cur = C->cur;
    int s, Ge;
    int64_t begin, end;
    sort_split(G, blk, C->n_slots[0], C->n_slots[1], s, Ge, begin, end);
    for (int i = tid; i <= nc; i += nt) h[i] = 0;
    __syncthreads();
    const float* X = bufsel(P.x, cur, s);
    // whole waves walk the range, kSortUnroll elements per thread with all loads issued first
    if (!P.sort_cells[s]) {
        unsigned c = 0;
        for (int64_t vb = begin; vb < end; vb += kSortUnroll * nt) {
            float x[kSortUnroll];
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                const int64_t v = vb + k * nt + tid;
                x[k] = v < end ? X[v] : -1.0f;
            }
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) c += x[k] > 0.0f ? 1u : 0u;
        }
        if (c) atomicAdd(&h[nc], c);
        __syncthreads();
        if (tid == 0) cnt[2 * nc + blk] = h[nc];
    } else {
        for (int64_t vb = begin; vb < end; vb += kSortUnroll * nt) {
            float x[kSortUnroll];
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                const int64_t v = vb + k * nt + tid;
                x[k] = v < end ? X[v] : -1.0f;
            }
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                int j = -1;
                if (x[k] > 0.0f) {
                    float w;
                    cell_of(x[k], nc, j, w);
                }
                wave_cell_add(h, j, false);
            }
        }
        __syncthreads();
        for (int i = tid; i < nc; i += nt)
            if (h[i]) atomicAdd(&cnt[s * nc + i], h[i]);
    }
}

__global__ void __launch_bounds__(1024) sort_count_kernel(Params P, unsigned* cnt) {
    extern __shared__ __align__(16) unsigned char smem[];
    sort_count_body(P, cnt, gridDim.x, blockIdx.x, smem);
}

// Exclusive scan of a[0..n) into o (one block of 1024 threads); a is cleared.  Returns the
// total to every thread.
__device__ unsigned block_excl_scan(unsigned* a, unsigned* o, int n, unsigned* sh) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (n + nt - 1) / nt;
    const int b = min(tid * per, n), e = min(b + per, n);
    unsigned sum = 0;
    for (int i = b; i < e; ++i) sum += a[i];
    sh[tid] = sum;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const unsigned t = tid >= off ? sh[tid - off] : 0u;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    unsigned run = sh[tid] - sum;
    for (int i = b; i < e; ++i) {
        o[i] = run;
        run += a[i];
        a[i] = 0;
    }
    const unsigned total = sh[nt - 1];
    __syncthreads();
    return total;
}

__device__ __forceinline__ void sort_scan_body(const Params& P, unsigned* cnt, unsigned* cursor, int G, unsigned* sh) {
    const int nc = P.n_cells;
    Ctrl* C = P.ctrl;
    int s, Ge;
    int64_t begin, end;
    sort_split(G, 0, C->n_slots[0], C->n_slots[1], s, Ge, begin, end);
    unsigned alive[2];
    for (int q = 0; q < 2; ++q) {
        if (P.sort_cells[q])
            alive[q] = block_excl_scan(cnt + q * nc, cursor + q * nc, nc, sh);
        else if (q == 0)
            alive[q] = block_excl_scan(cnt + 2 * nc, cursor + 2 * nc, Ge, sh);
        else
            alive[q] = block_excl_scan(cnt + 2 * nc + Ge, cursor + 2 * nc + Ge, G - Ge, sh);
    }
    if (threadIdx.x == 0) {
        C->sort_alive[0] = alive[0];
        C->sort_alive[1] = alive[1];
    }
}

__global__ void __launch_bounds__(1024) sort_scan_kernel(Params P, unsigned* cnt, unsigned* cursor, int G) {
    __shared__ unsigned sh[1024];
    sort_scan_body(P, cnt, cursor, G, sh);
}

__device__ __forceinline__ void sort_scatter_body(const Params& P, unsigned* cursor, int G, int blk,
                                                  unsigned char* smem) {
    const int nc = P.n_cells, tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    unsigned* h = reinterpret_cast<unsigned*>(smem);   // nc local counts, then cursors
    unsigned* base = h + nc;                            // nc reserved bases
    unsigned* wcnt = base + nc;                         // kSortUnroll x 16 wave counts
    unsigned* flag = wcnt + kSortUnroll * 16;
    Ctrl* C = P.ctrl;
    const unsigned cur = C->cur, nxt = cur ^ 1u;
    int s, Ge;
    int64_t begin, end;
    sort_split(G, blk, C->n_slots[0], C->n_slots[1], s, Ge, begin, end);
    const float* X = bufsel(P.x, cur, s);
    const float* VX = bufsel(P.vx, cur, s);
    const float* VY = bufsel(P.vy, cur, s);
    const float* VZ = bufsel(P.vz, cur, s);
    const uint32_t* ID = bufsel(P.id, cur, s);
    float* Xo = bufsel(P.x, nxt, s);
    float* VXo = bufsel(P.vx, nxt, s);
    float* VYo = bufsel(P.vy, nxt, s);
    float* VZo = bufsel(P.vz, nxt, s);
    uint32_t* IDo = bufsel(P.id, nxt, s);
    if (!P.sort_cells[s]) {
        // order-keeping compaction: this range's alive particles go, in order, to
        // [cursor[2 nc + b], ...); kSortUnroll chunks of blockDim elements per pair of
        // barriers, every load of the round issued first
        unsigned pos = cursor[2 * nc + blk];
        for (int64_t vb = begin; vb < end; vb += kSortUnroll * nt) {
            float x[kSortUnroll], vx[kSortUnroll], vy[kSortUnroll], vz[kSortUnroll];
            uint32_t id[kSortUnroll];
            unsigned long long m[kSortUnroll];
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                const int64_t v = vb + k * nt + tid;
                const bool in = v < end;
                x[k] = in ? X[v] : -1.0f;
                vx[k] = in ? VX[v] : 0.0f;
                vy[k] = in ? VY[v] : 0.0f;
                vz[k] = in ? VZ[v] : 0.0f;
                id[k] = in ? ID[v] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                m[k] = __ballot(x[k] > 0.0f);
                if (lane == 0) wcnt[k * 16 + wid] = (unsigned)__popcll(m[k]);
            }
            __syncthreads();
            unsigned off[kSortUnroll], run = 0;
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                unsigned before = 0, tot = 0;
                for (int w = 0; w < nw; ++w) {
                    const unsigned c = wcnt[k * 16 + w];
                    before += w < wid ? c : 0u;
                    tot += c;
                }
                off[k] = pos + run + before;
                run += tot;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                if (x[k] > 0.0f) {
                    const unsigned d = off[k] + (unsigned)__popcll(m[k] & ((1ull << lane) - 1ull));
                    Xo[d] = x[k];
                    VXo[d] = vx[k];
                    VYo[d] = vy[k];
                    VZo[d] = vz[k];
                    IDo[d] = id[k];
                }
            }
            pos += run;
        }
    } else {
        // cell sort: this block reserves, per cell, room after the blocks before it; whole
        // waves walk the range, and a wave's particles of one cell take consecutive places
        for (int i = tid; i < nc; i += nt) h[i] = 0;
        __syncthreads();
        for (int64_t vb = begin; vb < end; vb += kSortUnroll * nt) {
            float x[kSortUnroll];
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                const int64_t v = vb + k * nt + tid;
                x[k] = v < end ? X[v] : -1.0f;
            }
#pragma unroll
            for (int k = 0; k < kSortUnroll; ++k) {
                int j = -1;
                if (x[k] > 0.0f) {
                    float w;
                    cell_of(x[k], nc, j, w);
                }
                wave_cell_add(h, j, false);
            }
        }
        __syncthreads();
        for (int i = tid; i < nc; i += nt) {
            const unsigned c = h[i];
            base[i] = c ? atomicAdd(&cursor[s * nc + i], c) : 0u;
            h[i] = 0;
        }
        __syncthreads();
        for (int64_t vb = begin; vb < end; vb += 2 * nt) {
            float x[2], vx[2], vy[2], vz[2];
            uint32_t id[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t v = vb + k * nt + tid;
                const bool in = v < end;
                x[k] = in ? X[v] : -1.0f;
                vx[k] = in ? VX[v] : 0.0f;
                vy[k] = in ? VY[v] : 0.0f;
                vz[k] = in ? VZ[v] : 0.0f;
                id[k] = in ? ID[v] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                int j = -1;
                if (x[k] > 0.0f) {
                    float w;
                    cell_of(x[k], nc, j, w);
                }
                const unsigned r = wave_cell_add(h, j, true);
                if (j >= 0) {
                    const unsigned d = base[j] + r;
                    Xo[d] = x[k];
                    VXo[d] = vx[k];
                    VYo[d] = vy[k];
                    VZo[d] = vz[k];
                    IDo[d] = id[k];
                }
            }
        }
    }
    wait_memory_complete();
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = atomicAdd(&C->done, 1u);
        flag[0] = (prev == (unsigned)G - 1u) ? 1u : 0u;
    }
    __syncthreads();
    if (!flag[0] || tid != 0) return;
    C->n_slots[0] = (int64_t)ld_agent(&C->sort_alive[0]);
    C->n_slots[1] = (int64_t)ld_agent(&C->sort_alive[1]);
    C->cur = nxt;
    C->done = 0;
}

__global__ void __launch_bounds__(1024) sort_scatter_kernel(Params P, unsigned* cursor) {
    extern __shared__ __align__(16) unsigned char smem[];
    sort_scatter_body(P, cursor, gridDim.x, blockIdx.x, smem);
}

// The same three stages for several discharges at once: discharge k owns blocks
// [sseg[k], sseg[k + 1]) of the count and scatter launches and block k of the scan launch,
// and keeps its histograms in its own P.sort_cnt / P.sort_cursor.
__device__ __forceinline__ int batch_member(const int* seg, int nd, int b) {
    int lo = 0, hi = nd;   // seg[lo] <= b < seg[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(1024) sort_count_batch_kernel(const Params* __restrict__ batch,
                                                                const int* __restrict__ sseg, int nd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = batch_member(sseg, nd, blockIdx.x);
    const Params& P = batch[k];
    sort_count_body(P, P.sort_cnt, sseg[k + 1] - sseg[k], blockIdx.x - sseg[k], smem);
}

__global__ void __launch_bounds__(1024) sort_scan_batch_kernel(const Params* __restrict__ batch,
                                                               const int* __restrict__ sseg) {
    __shared__ unsigned sh[1024];
    const int k = blockIdx.x;
    const Params& P = batch[k];
    sort_scan_body(P, P.sort_cnt, P.sort_cursor, sseg[k + 1] - sseg[k], sh);
}

__global__ void __launch_bounds__(1024) sort_scatter_batch_kernel(const Params* __restrict__ batch,
                                                                  const int* __restrict__ sseg, int nd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = batch_member(sseg, nd, blockIdx.x);
    const Params& P = batch[k];
    sort_scatter_body(P, P.sort_cursor, sseg[k + 1] - sseg[k], blockIdx.x - sseg[k], smem);
}

// Moment window reset (kernel rather than a memset so it can sit in a captured graph).
__global__ void reset_window_kernel(Params P) {
    const int nn = P.n_cells + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 5 * nn; i += gridDim.x * blockDim.x) P.mom[i] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl* C = P.ctrl;
        C->n_samples = 0;
        C->n_steps_window = 0;
        C->n_periods = 0;
        C->J_period_max = 0.0;
        C->J_max_sum = 0.0;
        C->period_valid = (C->step % P.steps_per_period) == 0;
        for (int s = 0; s < 2; ++s)
            for (int e = 0; e < 2; ++e) C->absorbed_window[s][e] = 0;
    }
}

// ----------------------------------------------------------------------------------
// Launchers (called by the host library).
// ----------------------------------------------------------------------------------
#define PIC_PASS_SWITCH(KERNEL)                                                                                    \
    switch (mode) {                                                                                                \
        case kComplete | kAdvance | kRecord:                                                                       \
            hipLaunchKernelGGL(KERNEL<kComplete | kAdvance | kRecord>, dim3(blocks), dim3(threads), lds, st, P); \
            break;                                                                                                 \
        case kComplete | kRecord:                                                                                  \
            hipLaunchKernelGGL(KERNEL<kComplete | kRecord>, dim3(blocks), dim3(threads), lds, st, P);            \
            break;                                                                                                 \
        case kComplete | kAdvance:                                                                                 \
            hipLaunchKernelGGL(KERNEL<kComplete | kAdvance>, dim3(blocks), dim3(threads), lds, st, P);           \
            break;                                                                                                 \
        case kAdvance:                                                                                             \
            hipLaunchKernelGGL(KERNEL<kAdvance>, dim3(blocks), dim3(threads), lds, st, P);                       \
            break;                                                                                                 \
        case kComplete:                                                                                            \
            hipLaunchKernelGGL(KERNEL<kComplete>, dim3(blocks), dim3(threads), lds, st, P);                      \
            break;                                                                                                 \
        case kDeposit:                                                                                             \
            hipLaunchKernelGGL(KERNEL<kDeposit>, dim3(blocks), dim3(threads), lds, st, P);                       \
            break;                                                                                                 \
        default:                                                                                                   \
            return hipErrorInvalidValue;                                                                           \
    }

hipError_t launch_pass(int mode, const Params& P, int blocks, int threads, size_t lds, hipStream_t st, bool dyn) {
    if (dyn) {
        PIC_PASS_SWITCH(pass_dyn_kernel)
    } else {
        PIC_PASS_SWITCH(pass_kernel)
    }
    return hipGetLastError();
}

hipError_t launch_pass_batch(int mode, const Params* batch, const int* seg, int nd, int blocks, int threads,
                             size_t lds, hipStream_t st) {
    switch (mode) {
        case kComplete | kAdvance | kRecord:
            hipLaunchKernelGGL(pass_batch_kernel<kComplete | kAdvance | kRecord>, dim3(blocks), dim3(threads), lds,
                               st, batch, seg, nd);
            break;
        case kComplete | kRecord:
            hipLaunchKernelGGL(pass_batch_kernel<kComplete | kRecord>, dim3(blocks), dim3(threads), lds, st, batch,
                               seg, nd);
            break;
        case kComplete | kAdvance:
            hipLaunchKernelGGL(pass_batch_kernel<kComplete | kAdvance>, dim3(blocks), dim3(threads), lds, st, batch, seg,
                               nd);
            break;
        case kAdvance:
            hipLaunchKernelGGL(pass_batch_kernel<kAdvance>, dim3(blocks), dim3(threads), lds, st, batch, seg, nd);
            break;
        case kComplete:
            hipLaunchKernelGGL(pass_batch_kernel<kComplete>, dim3(blocks), dim3(threads), lds, st, batch, seg, nd);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t set_pass_batch_lds_limit(size_t bytes) {
    // The limit only grows, so that the launches of every live handle or batch stay within it.
    static std::mutex mu;
    static size_t limit = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (bytes <= limit) return hipSuccess;
    const int b = (int)bytes;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_batch_kernel<kComplete | kAdvance>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_batch_kernel<kAdvance>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_batch_kernel<kComplete>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_batch_kernel<kComplete | kAdvance | kRecord>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_batch_kernel<kComplete | kRecord>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess) limit = bytes;
    return e;
}

hipError_t pass_batch_occupancy(int threads, size_t lds, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pass_batch_kernel<kComplete | kAdvance>,
                                                        threads, lds);
}

hipError_t launch_load(const Params& P, int s, int64_t n, double vth, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(load_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, P, s, n, vth);
    return hipGetLastError();
}

// Staging for the warm-start tables of pic_load_profiles_noalloc, for callers that cannot
// allocate device memory: both species' tables of up to kNoAllocMaxPoints points, in
// device memory that lives as long as the process (one copy per GPU).  Host code reaches it
// only through the address noalloc_scratch returns, never through the array's name.
static __device__ __align__(256) double scratch[2 * 4 * kNoAllocMaxPoints];

// Address of this device's copy of scratch.  The first call on a device (with that device
// current) looks it up with hipGetSymbolAddress; later calls return the kept address.
hipError_t noalloc_scratch(int device, double** ptr, size_t* count) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *ptr = addr[device];
    *count = sizeof(scratch) / sizeof(double);
    return hipSuccess;
}

hipError_t launch_load_profile(const Params& P, int s, int64_t n, unsigned b, const double* tab, int np, double h_m,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (np < 2 || b > 1u) return hipErrorInvalidValue;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(load_profile_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, P, s, n, b, tab, np, h_m);
    return hipGetLastError();
}

size_t diag_lds_bytes(int nn, int n_bins) { return (size_t)6 * nn * sizeof(float) + (size_t)n_bins * sizeof(unsigned); }

hipError_t set_diag_lds_limit(size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&diag_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_diag(const Params& P, const DiagDev& D, int blocks, hipStream_t st) {
    if (blocks < 1 || D.n_bins < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_kernel, dim3(blocks), dim3(256), diag_lds_bytes(P.n_cells + 1, D.n_bins), st, P, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_nodes_kernel, dim3((P.n_cells + 256) / 256), dim3(256), 0, st, P, D);
    return hipGetLastError();
}

hipError_t launch_sort(const Params& P, unsigned* cnt, unsigned* cursor, int blocks, int threads, hipStream_t st) {
    if (blocks < 2 || blocks > kMaxSortBlocks || threads != 1024) return hipErrorInvalidValue;
    const size_t lds_count = (size_t)(P.n_cells + 1) * sizeof(unsigned);
    hipLaunchKernelGGL(sort_count_kernel, dim3(blocks), dim3(threads), lds_count, st, P, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, st, P, cnt, cursor, blocks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds_scatter = (size_t)2 * P.n_cells * sizeof(unsigned) + (kSortUnroll * 16 + 1) * sizeof(unsigned);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(blocks), dim3(threads), lds_scatter, st, P, cursor);
    return hipGetLastError();
}

hipError_t launch_sort_batch(const Params* batch, const int* sseg, int nd, int blocks, int max_cells,
                             hipStream_t st) {
    if (nd < 1 || blocks < 2 * nd || max_cells < 1) return hipErrorInvalidValue;
    const size_t lds_count = (size_t)(max_cells + 1) * sizeof(unsigned);
    hipLaunchKernelGGL(sort_count_batch_kernel, dim3(blocks), dim3(1024), lds_count, st, batch, sseg, nd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scan_batch_kernel, dim3(nd), dim3(1024), 0, st, batch, sseg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds_scatter = (size_t)2 * max_cells * sizeof(unsigned) + (kSortUnroll * 16 + 1) * sizeof(unsigned);
    hipLaunchKernelGGL(sort_scatter_batch_kernel, dim3(blocks), dim3(1024), lds_scatter, st, batch, sseg, nd);
    return hipGetLastError();
}

hipError_t launch_reset_window(const Params& P, hipStream_t st) {
    hipLaunchKernelGGL(reset_window_kernel, dim3(8), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t pass_occupancy(int threads, size_t lds, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pass_kernel<kComplete | kAdvance>, threads, lds);
}

hipError_t set_pass_lds_limit(size_t bytes) {
    // The limit only grows, so that the launches of every live handle or batch stay within it.
    static std::mutex mu;
    static size_t limit = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (bytes <= limit) return hipSuccess;
    const int b = (int)bytes;
    const void* kernels[] = {
        reinterpret_cast<const void*>(&pass_kernel<kComplete | kAdvance>),
        reinterpret_cast<const void*>(&pass_kernel<kAdvance>),
        reinterpret_cast<const void*>(&pass_kernel<kComplete>),
        reinterpret_cast<const void*>(&pass_kernel<kDeposit>),
        reinterpret_cast<const void*>(&pass_kernel<kComplete | kAdvance | kRecord>),
        reinterpret_cast<const void*>(&pass_kernel<kComplete | kRecord>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kComplete | kAdvance>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kAdvance>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kComplete>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kDeposit>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kComplete | kAdvance | kRecord>),
        reinterpret_cast<const void*>(&pass_dyn_kernel<kComplete | kRecord>)};
    hipError_t e = hipSuccess;
    for (const void* k : kernels)
        if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e == hipSuccess) limit = bytes;
    return e;
}

}  // namespace pic
