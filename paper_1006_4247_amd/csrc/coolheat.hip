// Cooling / heating replica exchange (paper Sec. III.B).
//
// Site map (spin s, field S of the other sublattice, k = eps |S|, cos(theta) = s.S/|S|):
// cooling turns s towards S by alpha = eps |p| = k sin(theta), p = S - (S.s) s,
//     s' = s cos(alpha) + (p/|p|) sin(alpha),   theta' = theta - alpha,
// a bijection of the sphere for k < 1 with Jacobian
//     (1 - k cos(theta)) (cos(alpha) - cos(theta) k sinc(alpha)).
// Heating inverts it: theta from theta' by Newton's method on
// theta - k sin(theta) = theta', then s = s' cos(alpha) - (q/|q|) sin(alpha),
// q = S - (S.s') s'.  Lattice cooling C maps parity 0 (fields from parity 1) and then
// parity 1; heating C^-1 undoes parity 1 and then parity 0.
//
// Exchange of x at b1 = beta_i and y at b2 = beta_{i+1}: the involution
// (x, y) -> (C^-1 y at b1, C x at b2) is accepted iff ln u < ln A,
//     ln A = b1 H(x) + b2 H(y) - b1 H(C^-1 y) - b2 H(C x) + ln det J_C(x) - ln det J_C(C^-1 y).
// Legs: one workgroup cools x, one heats y, into the candidate buffer, with the log
// Jacobian (FP64 sum of site terms) and the fused FP64 energy; a per-chain kernel
// decides; accepted candidates are copied back.  A site with k >= 1 makes the pair's
// Jacobian NaN (the map is not a bijection): the pair is rejected and guard bit 8 set.
#include "hsg_device.h"
#include "hsg_launch.h"

namespace hsg {

constexpr int kChThreads = 256;

__device__ __forceinline__ double ch_sinc(double a) {
    return fabs(a) < 1e-4 ? 1.0 - a * a / 6.0 : sin(a) / a;
}

// log Jacobian of cooling at a spin with cos(theta) = c, sin(theta) = st
__device__ __forceinline__ double cool_log_jac(double c, double st, double k) {
    const double alpha = k * st;
    return log(1.0 - k * c) + log(cos(alpha) - c * k * ch_sinc(alpha));
}

template <typename T>
__device__ __forceinline__ T d_atan2(T y, T x);
template <>
__device__ __forceinline__ float d_atan2(float y, float x) { return atan2f(y, x); }
template <>
__device__ __forceinline__ double d_atan2(double y, double x) { return atan2(y, x); }

// Binary32 helpers: sine and cosine of x radians from the hardware sine/cosine in
// turns (|error| < 1.3e-7 for |x| <= 2 pi), and the site log Jacobian as one
// logarithm of the product of its two factors (absolute error ~1e-7 per site; the
// sum over sites is FP64).
__device__ __forceinline__ void sincos_hw(float x, float& s, float& c) {
    const float t = x * 0.159154943091895336f;
    s = __builtin_amdgcn_sinf(t);
    c = __builtin_amdgcn_cosf(t);
}

__device__ __forceinline__ float cool_log_jac_f(float c, float k, float alpha, float sa, float ca) {
    const float sinc = alpha < 1e-3f ? fmaf(-alpha * alpha, 1.0f / 6.0f, 1.0f) : sa / alpha;
    return 0.693147180559945309f * __builtin_amdgcn_logf(fmaf(-k, c, 1.0f) * fmaf(-c * k, sinc, ca));
}

// Binary32 site map (same steps as the generic one below, hardware sine/cosine).
template <bool HEAT>
__device__ __forceinline__ double coolheat_site_f(float& sx, float& sy, float& sz, float Sx, float Sy, float Sz,
                                                  float eps) {
    const float nS = sqrtf(fmaf(Sz, Sz, fmaf(Sy, Sy, Sx * Sx)));
    const float k = eps * nS;
    if (!(k < 1.0f)) return __builtin_nan("");
    if (nS == 0.0f) return 0.0;
    const float Ss = fmaf(Sz, sz, fmaf(Sy, sy, Sx * sx));
    const float px = fmaf(-Ss, sx, Sx), py = fmaf(-Ss, sy, Sy), pz = fmaf(-Ss, sz, Sz);
    const float np = sqrtf(fmaf(pz, pz, fmaf(py, py, px * px)));
    float alpha, c;
    if (!HEAT) {
        alpha = eps * np;
        c = Ss / nS;
    } else {
        const float thp = atan2f(np, Ss);  // theta' in [0, pi]
        float sn, cs;
        sincos_hw(thp, sn, cs);
        float th = fmaf(k, sn, thp);
        for (int it = 0; it < 8; ++it) {
            sincos_hw(th, sn, cs);
            const float d = (fmaf(-k, sn, th) - thp) / fmaf(-k, cs, 1.0f);
            th -= d;
            if (!(fabsf(d) > 1e-7f * (1.0f + th))) break;
        }
        sincos_hw(th, sn, cs);
        alpha = th - thp;
        c = cs;
    }
    float sa, ca;
    sincos_hw(alpha, sa, ca);
    if (np > 0.0f) {
        const float f = (HEAT ? -sa : sa) / np;
        sx = fmaf(px, f, sx * ca);
        sy = fmaf(py, f, sy * ca);
        sz = fmaf(pz, f, sz * ca);
    }
    return static_cast<double>(cool_log_jac_f(c, k, alpha, sa, ca));
}

// One site: cool (HEAT = false) or heat s in place given the field; returns the log
// Jacobian of cooling (at s before cooling / at the heated result), NaN if k >= 1.
template <typename T, bool HEAT>
__device__ __forceinline__ double coolheat_site(T& sx, T& sy, T& sz, T Sx, T Sy, T Sz, T eps) {
    if constexpr (sizeof(T) == 4) return coolheat_site_f<HEAT>(sx, sy, sz, Sx, Sy, Sz, eps);
    const T nS = sqrt(fma(Sz, Sz, fma(Sy, Sy, Sx * Sx)));
    const T k = eps * nS;
    if (!(k < T(1))) return __builtin_nan("");
    if (nS == T(0)) return 0.0;
    const T Ss = fma(Sz, sz, fma(Sy, sy, Sx * sx));
    const T px = fma(-Ss, sx, Sx), py = fma(-Ss, sy, Sy), pz = fma(-Ss, sz, Sz);
    const T np = sqrt(fma(pz, pz, fma(py, py, px * px)));
    if (!HEAT) {
        const T alpha = eps * np;
        const T ca = cos(alpha), sa = sin(alpha);
        if (np > T(0)) {
            const T f = sa / np;
            sx = fma(px, f, sx * ca);
            sy = fma(py, f, sy * ca);
            sz = fma(pz, f, sz * ca);
        }
        return cool_log_jac(static_cast<double>(Ss) / static_cast<double>(nS),
                            static_cast<double>(np) / static_cast<double>(nS), static_cast<double>(k));
    } else {
        const T thp = d_atan2<T>(np, Ss);  // theta' in [0, pi]
        T th = fma(k, sin(thp), thp);
        for (int it = 0; it < 50; ++it) {
            const T g = fma(-k, sin(th), th) - thp;
            const T d = g / fma(-k, cos(th), T(1));
            th -= d;
            if (!(fabs(d) > T(sizeof(T) == 4 ? 1e-7 : 1e-16) * (T(1) + th))) break;
        }
        const T alpha = th - thp;
        const T ca = cos(alpha), sa = sin(alpha);
        if (np > T(0)) {
            const T f = -sa / np;
            sx = fma(px, f, sx * ca);
            sy = fma(py, f, sy * ca);
            sz = fma(pz, f, sz * ca);
        }
        const double thd = static_cast<double>(th);
        return cool_log_jac(cos(thd), sin(thd), static_cast<double>(k));
    }
}

// Work item b of a launch over the pairs i = i0 + istep m (m < npc) of every chain,
// two legs each: leg 0 cools the configuration at beta_i, leg 1 heats the one at
// beta_{i+1}.
struct ChItem {
    int ch, i, leg, slot;
};

__device__ __forceinline__ ChItem ch_item(const hsg_ensemble& e, int b, int i0, int istep, int npc) {
    ChItem it;
    const int R = e.n_temps;
    it.ch = b / (2 * npc);
    const int rest = b - it.ch * 2 * npc;
    it.leg = rest & 1;
    it.i = i0 + istep * (rest >> 1);
    it.slot = it.ch * R + label(e.slot_of_temp[it.ch * R + it.i + it.leg], R, e.guard);
    return it;
}

__device__ void coolheat_decide_chain(const hsg_ensemble& e, int ch, int i0, int istep, int npc, int last,
                                      int* cp);

// The map parameter: one for every pair, or pair i's own from a device array
// (pair != nullptr).
struct ChEps {
    double eps;
    const double* pair;
};

template <typename T>
__device__ __forceinline__ T ch_eps(const ChEps& c, int i) {
    return static_cast<T>(c.pair ? c.pair[i] : c.eps);
}

// LDS-resident legs (L <= 16): the replica in LDS, couplings from global memory.
// NT threads: 256 where a launch holds many pairs, more for the single pair per
// chain of an ascending round, whose legs then finish sooner.
//
// PREV (ascending rounds i0 >= 1, one pair per chain): the cooling leg's workgroup
// first decides pair i0 - 1 of its chain and copies that pair's accepted candidates
// over their spins, then cools the configuration the decision left at beta_{i0}
// (read from the candidate buffer if the exchange was accepted).  Only that leg
// depends on pair i0 - 1; the heating leg takes the configuration at beta_{i0+1},
// which pair i0 - 1 does not touch, and runs meanwhile.
//
// HEATALL (ascending passes in two launches, see k_coolheat_cool_chain): work item b
// heats, for pair i = b mod (R - 1) of chain b / (R - 1), the configuration at
// beta_{i+1} as the pass finds it — no pair before i touches that temperature, so the
// heating legs of all pairs run at once, before any decision.
template <typename T, int L, int NT, bool PREV, bool HEATALL = false>
__global__ void __launch_bounds__(NT) k_coolheat_leg_res(hsg_ensemble e, ChEps ce, int i0, int istep, int npc) {
    constexpr int N = L * L * L, NH = N / 2;
    constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sh = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[NT / 64];
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    T* cand = reinterpret_cast<T*>(scr + sl.cand);
    T* spins = static_cast<T*>(e.spins);
    ChItem it;
    bool from_cand = false;
    if constexpr (PREV) {
        __shared__ int s_prev[3];
        const int R = e.n_temps;
        it.ch = static_cast<int>(blockIdx.x) >> 1;
        it.leg = static_cast<int>(blockIdx.x) & 1;
        it.i = i0;
        if (it.leg == 0) {  // uniform over the workgroup
            if (threadIdx.x == 0) {
                coolheat_decide_chain(e, it.ch, i0 - 1, 1, 1, 0, s_prev);
                s_prev[2] = label(e.slot_of_temp[it.ch * R + i0], R, e.guard);
            }
            __syncthreads();
            it.slot = it.ch * R + s_prev[2];
            from_cand = s_prev[0] >= 0;  // then s_prev[2] == s_prev[0]
            if (s_prev[1] >= 0) {        // C^-1 y, now at beta_{i0-1}, back over its spins
                const size_t y = static_cast<size_t>(it.ch) * R + s_prev[1];
                const uint4* cs = reinterpret_cast<const uint4*>(cand + y * 3 * N);
                uint4* cd = reinterpret_cast<uint4*>(spins + y * 3 * N);
                for (int v = threadIdx.x; v < NV; v += NT) cd[v] = cs[v];
            }
        } else {
            it.slot = it.ch * R + label(e.slot_of_temp[it.ch * R + i0 + 1], R, e.guard);
        }
    } else if constexpr (HEATALL) {
        const int R = e.n_temps;
        it.ch = static_cast<int>(blockIdx.x) / (R - 1);
        it.i = static_cast<int>(blockIdx.x) - it.ch * (R - 1);
        it.leg = 1;
        it.slot = it.ch * R + label(e.slot_of_temp[it.ch * R + it.i + 1], R, e.guard);
    } else {
        it = ch_item(e, blockIdx.x, i0, istep, npc);
    }
    const T eps = ch_eps<T>(ce, it.i);
    const int smp = it.ch / e.n_chains;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* own = spins + static_cast<size_t>(it.slot) * 3 * N;
    uint4* dst = reinterpret_cast<uint4*>(cand + static_cast<size_t>(it.slot) * 3 * N);
    uint4* s4 = reinterpret_cast<uint4*>(sh);
    if (from_cand) {  // C x of pair i0 - 1: into LDS and back over the spins of its slot
        uint4* back = reinterpret_cast<uint4*>(own);
        for (int v = threadIdx.x; v < NV; v += NT) {
            const uint4 a = dst[v];
            s4[v] = a;
            back[v] = a;
        }
    } else {
        const uint4* src = reinterpret_cast<const uint4*>(own);
        for (int v = threadIdx.x; v < NV; v += NT) s4[v] = src[v];
    }
    __syncthreads();
    double ld = 0.0, en = 0.0;
    for (int step = 0; step < 2; ++step) {
        const int p = it.leg ? 1 - step : step;
        const T* o0 = sh + (0 * 2 + (1 - p)) * NH;
        const T* o1 = sh + (1 * 2 + (1 - p)) * NH;
        const T* o2 = sh + (2 * 2 + (1 - p)) * NH;
        T* w0 = sh + (0 * 2 + p) * NH;
        T* w1 = sh + (1 * 2 + p) * NH;
        T* w2 = sh + (2 * 2 + p) * NH;
#pragma unroll  // the sites of a thread are independent: their latency chains interleave
        for (int h = threadIdx.x; h < NH; h += NT) {
            const Nbr nb = neighbours<L>(h, p, L);
            T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int mu = d >> 1;
                const T jj = (d & 1) ? J[(mu * 2 + (1 - p)) * NH + nb.n[d]] : J[(mu * 2 + p) * NH + h];
                const int idx = nb.n[d];
                Sx = fma(jj, o0[idx], Sx);
                Sy = fma(jj, o1[idx], Sy);
                Sz = fma(jj, o2[idx], Sz);
            }
            T sx = w0[h], sy = w1[h], sz = w2[h];
            ld += it.leg ? coolheat_site<T, true>(sx, sy, sz, Sx, Sy, Sz, eps)
                         : coolheat_site<T, false>(sx, sy, sz, Sx, Sy, Sz, eps);
            w0[h] = sx;
            w1[h] = sy;
            w2[h] = sz;
            if (step == 1) {
                const double dx = sx, dy = sy, dz = sz;
                en += fma(dz, static_cast<double>(Sz), fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
            }
        }
        __syncthreads();
    }
    for (int v = threadIdx.x; v < NV; v += NT) dst[v] = s4[v];
    const double LD = block_sum<NT>(ld, red);
    const double H = -block_sum<NT>(en, red);
    if (threadIdx.x == 0) {
        e.work[(static_cast<size_t>(it.ch) * (e.n_temps - 1) + it.i) * 2 + it.leg] = LD;
        reinterpret_cast<double*>(scr + sl.cand_energy)[it.slot] = H;
        if (isnan(LD)) atomicOr(e.guard, 8);
    }
}

// Generic legs (any even L): the candidate in global memory.  NT threads: 256 where a
// launch holds many pairs, more for the single pair per chain of an ascending round.
// PREV as for the LDS-resident legs: the cooling workgroup first decides and copies
// pair i0 - 1; where that exchange was accepted, the configuration at beta_{i0} already
// sits in this slot's candidate buffer and is copied back over its spins before the
// map overwrites it.
template <typename T, int NT, bool PREV>
__global__ void __launch_bounds__(NT) k_coolheat_leg(hsg_ensemble e, ChEps ce, int i0, int istep, int npc) {
    __shared__ double red[NT / 64];
    const int L = e.L, N = L * L * L, NH = N / 2;
    const int nv = 3 * N * static_cast<int>(sizeof(T)) / 16;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    T* cand = reinterpret_cast<T*>(scr + sl.cand);
    T* spins = static_cast<T*>(e.spins);
    ChItem it;
    bool from_cand = false;
    if constexpr (PREV) {
        __shared__ int s_prev[3];
        const int R = e.n_temps;
        it.ch = static_cast<int>(blockIdx.x) >> 1;
        it.leg = static_cast<int>(blockIdx.x) & 1;
        it.i = i0;
        if (it.leg == 0) {  // uniform over the workgroup
            if (threadIdx.x == 0) {
                coolheat_decide_chain(e, it.ch, i0 - 1, 1, 1, 0, s_prev);
                s_prev[2] = label(e.slot_of_temp[it.ch * R + i0], R, e.guard);
            }
            __syncthreads();
            it.slot = it.ch * R + s_prev[2];
            from_cand = s_prev[0] >= 0;  // then s_prev[2] == s_prev[0]
            if (s_prev[1] >= 0) {        // C^-1 y, now at beta_{i0-1}, back over its spins
                const size_t y = static_cast<size_t>(it.ch) * R + s_prev[1];
                const uint4* cs = reinterpret_cast<const uint4*>(cand + y * 3 * N);
                uint4* cd = reinterpret_cast<uint4*>(spins + y * 3 * N);
                for (int v = threadIdx.x; v < nv; v += NT) cd[v] = cs[v];
            }
        } else {
            it.slot = it.ch * R + label(e.slot_of_temp[it.ch * R + i0 + 1], R, e.guard);
        }
    } else {
        it = ch_item(e, blockIdx.x, i0, istep, npc);
    }
    const T eps = ch_eps<T>(ce, it.i);
    const int smp = it.ch / e.n_chains;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* c = cand + static_cast<size_t>(it.slot) * 3 * N;
    {
        uint4* cv = reinterpret_cast<uint4*>(c);
        uint4* sv = reinterpret_cast<uint4*>(spins + static_cast<size_t>(it.slot) * 3 * N);
        if (from_cand)  // C x of pair i0 - 1 becomes its slot's spins; the map starts from it
            for (int v = threadIdx.x; v < nv; v += NT) sv[v] = cv[v];
        else
            for (int v = threadIdx.x; v < nv; v += NT) cv[v] = sv[v];
    }
    __syncthreads();
    double ld = 0.0, en = 0.0;
    for (int step = 0; step < 2; ++step) {
        const int p = it.leg ? 1 - step : step;
        const T* o0 = c + (0 * 2 + (1 - p)) * NH;
        const T* o1 = c + (1 * 2 + (1 - p)) * NH;
        const T* o2 = c + (2 * 2 + (1 - p)) * NH;
        T* w0 = c + (0 * 2 + p) * NH;
        T* w1 = c + (1 * 2 + p) * NH;
        T* w2 = c + (2 * 2 + p) * NH;
        for (int h = threadIdx.x; h < NH; h += NT) {
            const Nbr nb = neighbours<0>(h, p, L);
            T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int mu = d >> 1;
                const T jj = (d & 1) ? J[(mu * 2 + (1 - p)) * NH + nb.n[d]] : J[(mu * 2 + p) * NH + h];
                const int idx = nb.n[d];
                Sx = fma(jj, o0[idx], Sx);
                Sy = fma(jj, o1[idx], Sy);
                Sz = fma(jj, o2[idx], Sz);
            }
            T sx = w0[h], sy = w1[h], sz = w2[h];
            ld += it.leg ? coolheat_site<T, true>(sx, sy, sz, Sx, Sy, Sz, eps)
                         : coolheat_site<T, false>(sx, sy, sz, Sx, Sy, Sz, eps);
            w0[h] = sx;
            w1[h] = sy;
            w2[h] = sz;
            if (step == 1) {
                const double dx = sx, dy = sy, dz = sz;
                en += fma(dz, static_cast<double>(Sz), fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
            }
        }
        __syncthreads();  // the next half-step reads this one's spins
    }
    const double LD = block_sum<NT>(ld, red);
    const double H = -block_sum<NT>(en, red);
    if (threadIdx.x == 0) {
        e.work[(static_cast<size_t>(it.ch) * (e.n_temps - 1) + it.i) * 2 + it.leg] = LD;
        reinterpret_cast<double*>(scr + sl.cand_energy)[it.slot] = H;
        if (isnan(LD)) atomicOr(e.guard, 8);
    }
}

// Decision of pair i of chain ch with exchange counter n: cp[leg] receives the slot
// whose candidate replaces its spins, or -1.
__device__ __forceinline__ void coolheat_decide_pair(const hsg_ensemble& e, int ch, int i, uint32_t n, int* cp) {
    const int R = e.n_temps;
    const ScratchLayout sl = scratch_layout(e);
    const double* cen = reinterpret_cast<const double*>(static_cast<unsigned char*>(e.scratch) + sl.cand_energy) +
                        static_cast<size_t>(ch) * R;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    double* en = e.energy + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const double* W = e.work + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const int x = label(sot[i], R, e.guard), y = label(sot[i + 1], R, e.guard);
    const double b1 = e.betas[i], b2 = e.betas[i + 1];
    const double lnA = b1 * en[x] + b2 * en[y] - b1 * cen[y] - b2 * cen[x] + W[2 * i] - W[2 * i + 1];
    const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, key_lo(e.seed), key_hi(e.seed));
    st[2 * i] += 1;
    const bool ok = log(u01_52(w.w0, w.w1)) < lnA;
    cp[0] = ok ? x : -1;
    cp[1] = ok ? y : -1;
    if (ok) {
        en[x] = cen[x];
        en[y] = cen[y];
        sot[i] = y;
        sot[i + 1] = x;
        tos[x] = i + 1;
        tos[y] = i;
        st[2 * i + 1] += 1;
    }
}

// After the last decision of a call: clear the diagnostics of the pairs not attempted
// (even / odd pairs), advance the exchange counter and update the round trips.
__device__ __forceinline__ void coolheat_finish_chain(const hsg_ensemble& e, int ch, int i0, int istep) {
    const int R = e.n_temps;
    double* W = e.work + static_cast<size_t>(ch) * (R - 1) * 2;
    if (istep == 2)
        for (int i = 1 - (i0 & 1); i < R - 1; i += 2) {
            W[2 * i] = 0.0;
            W[2 * i + 1] = 0.0;
        }
    e.swap_ctr[ch] += 1u;
    const int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* rs = e.rt_state + static_cast<size_t>(ch) * R;
    long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + static_cast<size_t>(ch) * R;
    for (int r = 0; r < R; ++r) {
        const int Tr = tos[r];
        if (Tr == 0) {
            if (rs[r] == 2) rtt[r] += 1;
            rs[r] = 1;
        } else if (Tr == R - 1) {
            if (rs[r] == 1) rs[r] = 2;
        }
    }
}

// Decisions of the pairs i0 + istep m (m < npc) of chain ch, in order; `last` finishes
// the call.  cp[2 m + leg] receives the slot whose candidate replaces its spins, or -1.
__device__ void coolheat_decide_chain(const hsg_ensemble& e, int ch, int i0, int istep, int npc, int last,
                                      int* cp) {
    const uint32_t n = e.swap_ctr[ch];
    for (int m = 0; m < npc; ++m) coolheat_decide_pair(e, ch, i0 + istep * m, n, cp + 2 * m);
    if (last) coolheat_finish_chain(e, ch, i0, istep);
}

// Even or odd pairs: one thread per (chain, pair), the pairs of a call being disjoint;
// entry (chain, m, leg) of the flags array names the slot whose candidate replaces its
// spins, or -1.  The copy-back launch finishes each chain.
__global__ void k_coolheat_decide(hsg_ensemble e, int i0, int istep, int npc) {
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= e.n_samples * e.n_chains * npc) return;
    const int ch = t / npc, m = t - ch * npc;
    const ScratchLayout sl = scratch_layout(e);
    int* flags = reinterpret_cast<int*>(static_cast<unsigned char*>(e.scratch) + sl.flags);
    coolheat_decide_pair(e, ch, i0 + istep * m, e.swap_ctr[ch], flags + static_cast<size_t>(t) * 2);
}

// Ascending rounds (pair i of every chain): one workgroup per chain decides its pair
// and copies the accepted candidates over the spins of their slots.  While thread 0
// decides, every thread loads the first kPre vectors of its share of both candidates
// (a 16^3 binary32 replica entirely), so the copy's loads overlap the decision.
constexpr int kDecideCopyThreads = 512;
constexpr int kPre = 6;

template <typename T>
__global__ void __launch_bounds__(kDecideCopyThreads) k_coolheat_decide_copy(hsg_ensemble e, int i, int istep,
                                                                             int last) {
    __shared__ int s_slot[2];
    const int ch = static_cast<int>(blockIdx.x);
    const int R = e.n_temps;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const int nv = static_cast<int>(3 * N * sizeof(T) / 16);
    const int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    // the pair's slots before the decision: x at beta_i (leg 0), y at beta_{i+1} (leg 1)
    const int xy[2] = {label(sot[i], R, e.guard), label(sot[i + 1], R, e.guard)};
    __syncthreads();  // every thread holds them before thread 0 may swap the labels
    uint4 pre[2][kPre];
#pragma unroll
    for (int leg = 0; leg < 2; ++leg) {
        const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const T*>(scr + sl.cand) +
                                                          (static_cast<size_t>(ch) * R + xy[leg]) * 3 * N);
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int v = static_cast<int>(threadIdx.x) + k * kDecideCopyThreads;
            pre[leg][k] = v < nv ? src[v] : make_uint4(0, 0, 0, 0);
        }
    }
    if (threadIdx.x == 0) coolheat_decide_chain(e, ch, i, istep, 1, last, s_slot);
    __syncthreads();
#pragma unroll
    for (int leg = 0; leg < 2; ++leg) {
        if (s_slot[leg] < 0) continue;  // uniform over the workgroup; else s_slot[leg] == xy[leg]
        const size_t slot = static_cast<size_t>(ch) * R + xy[leg];
        const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const T*>(scr + sl.cand) + slot * 3 * N);
        uint4* dst = reinterpret_cast<uint4*>(static_cast<T*>(e.spins) + slot * 3 * N);
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int v = static_cast<int>(threadIdx.x) + k * kDecideCopyThreads;
            if (v < nv) dst[v] = pre[leg][k];
        }
        for (int v = static_cast<int>(threadIdx.x) + kPre * kDecideCopyThreads; v < nv; v += kDecideCopyThreads)
            dst[v] = src[v];
    }
}

// Workgroup b copies candidate b of the decided pairs ((chain, m, leg) order), if
// accepted, over the spins of its slot.
template <typename T>
__global__ void k_coolheat_copyback(hsg_ensemble e, int i0, int istep, int npc) {
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const int ch = static_cast<int>(blockIdx.x) / (2 * npc);
    if (static_cast<int>(blockIdx.x) % (2 * npc) == 0 && threadIdx.x == 0) coolheat_finish_chain(e, ch, i0, istep);
    const int r = reinterpret_cast<const int*>(scr + sl.flags)[blockIdx.x];
    if (r < 0) return;
    const size_t slot = static_cast<size_t>(ch) * e.n_temps + r;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const T*>(scr + sl.cand) + slot * 3 * N);
    uint4* dst = reinterpret_cast<uint4*>(static_cast<T*>(e.spins) + slot * 3 * N);
    const size_t nv = 3 * N * sizeof(T) / 16;
    for (size_t v = threadIdx.x; v < nv; v += blockDim.x) dst[v] = src[v];
}

// A call that selects no pair: only the per-chain finish.
__global__ void k_coolheat_finish(hsg_ensemble e, int i0, int istep) {
    const int ch = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (ch < e.n_samples * e.n_chains) coolheat_finish_chain(e, ch, i0, istep);
}

// Ascending binary32 pass, second launch (the first heats the configuration at
// beta_{i+1} for every pair i at once, HEATALL legs): one workgroup per chain walks
// the pairs.  The configuration at beta_i sits in LDS; the workgroup cools it (the
// cooling legs' arithmetic, thread mapping and reductions) and decides the pair with
// the decision kernels' formula, from copies in LDS of the chain's labels, energies,
// statistics, temperatures and of the heating legs' results, with the decision
// uniforms drawn up front (the decision then waits for no memory round trip; its
// results go out as stores).  An accepted pair writes the cooled configuration, now at
// beta_{i+1}, over its slot and the heated one over the other slot (its vectors were
// requested into registers when the pair began); the cooled configuration stays in LDS
// as the next pair's lower one.  A rejected pair leaves the next pair's lower
// configuration where pair i's upper one was: its planes were requested from HBM
// straight into a second LDS buffer (loads that bypass the registers) when pair i
// began.  The chain's couplings sit in LDS for the whole pass; barriers are LDS-only
// so that those loads stay in flight until the wait before the decision.  Results
// equal the per-pair launches' bit for bit.
constexpr int kChainMaxPairs = 128;

template <int L, int NT>
__global__ void __launch_bounds__(NT) k_coolheat_cool_chain(hsg_ensemble e, ChEps ce) {
    using T = float;
    constexpr int N = L * L * L, NH = N / 2;
    constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per replica
    constexpr int PC = (NV + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Js = reinterpret_cast<T*>(smem_raw);  // [3][2][NH]
    T* bufs = Js + 3 * N;                    // two replicas [3][2][NH]
    __shared__ double red[2 * (NT / 64)];
    __shared__ double s_en[kChainMaxPairs + 1], s_cen[kChainMaxPairs + 1], s_beta[kChainMaxPairs + 1];
    __shared__ double s_wh[kChainMaxPairs], s_logu[kChainMaxPairs];
    __shared__ long long s_st[2 * kChainMaxPairs];
    __shared__ int s_sot[kChainMaxPairs + 1];
    __shared__ int s_ok;
    const int R = e.n_temps;
    const int ch = static_cast<int>(blockIdx.x);
    const int t = static_cast<int>(threadIdx.x);
    const int smp = ch / e.n_chains;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const T* cand = reinterpret_cast<const T*>(scr + sl.cand);
    double* cen = reinterpret_cast<double*>(scr + sl.cand_energy) + static_cast<size_t>(ch) * R;
    T* spins = static_cast<T*>(e.spins);
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    double* en = e.energy + static_cast<size_t>(ch) * R;
    double* W = e.work + static_cast<size_t>(ch) * (R - 1) * 2;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    for (int r = t; r < R; r += NT) {
        s_sot[r] = label(sot[r], R, e.guard);
        s_en[r] = en[r];
        s_cen[r] = cen[r];  // the heated configurations' energies, by slot
        s_beta[r] = e.betas[r];
    }
    for (int i = t; i < R - 1; i += NT) {
        s_wh[i] = W[2 * i + 1];
        const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, key_lo(e.seed), key_hi(e.seed));
        s_logu[i] = log(u01_52(w.w0, w.w1));
        s_st[2 * i] = st[2 * i];
        s_st[2 * i + 1] = st[2 * i + 1];
    }
    __syncthreads();
    int xs = s_sot[0];  // slot of the configuration at beta_i
    {
        const uint4* js = reinterpret_cast<const uint4*>(static_cast<const T*>(e.couplings) +
                                                         static_cast<size_t>(smp) * 3 * N);
        const uint4* xv = reinterpret_cast<const uint4*>(spins + (static_cast<size_t>(ch) * R + xs) * 3 * N);
        uint4* jd = reinterpret_cast<uint4*>(Js);
        uint4* xd = reinterpret_cast<uint4*>(bufs);
        for (int v = t; v < NV; v += NT) {
            jd[v] = js[v];
            xd[v] = xv[v];
        }
    }
    __syncthreads();
    int cur = 0;
    for (int i = 0; i < R - 1; ++i) {
        // the configuration at beta_{i+1}: pairs before i never touch it
        const int ys = s_sot[i + 1];
        const T eps = ch_eps<T>(ce, i);
        T* sh = bufs + static_cast<size_t>(cur) * 3 * N;
        T* other = bufs + static_cast<size_t>(1 - cur) * 3 * N;
        const size_t gy = static_cast<size_t>(ch) * R + ys;
        uint4 hv[PC];  // the heated candidate, copied over slot ys if the pair is accepted
        {
            const uint4* cy = reinterpret_cast<const uint4*>(cand + gy * 3 * N);
#pragma unroll
            for (int k = 0; k < PC; ++k) {
                const int v = t + k * NT;
                hv[k] = v < NV ? cy[v] : make_uint4(0, 0, 0, 0);
            }
        }
        if (i + 2 < R) {  // its planes, the next lower configuration should pair i be rejected
            const uint4* src = reinterpret_cast<const uint4*>(spins + gy * 3 * N);
            uint4* dst = reinterpret_cast<uint4*>(other);
            const int wave_base = t & ~63;
            for (int v0 = wave_base; v0 < NV; v0 += NT) {
                const int v = v0 + (t & 63);
                if (v < NV)
                    __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + v),
                                                     (__attribute__((address_space(3))) void*)(dst + v0), 16, 0, 0);
            }
        }
        double ld = 0.0, en_acc = 0.0;
        for (int step = 0; step < 2; ++step) {
            const int p = step;  // cooling maps parity 0, then parity 1
            const T* o0 = sh + (0 * 2 + (1 - p)) * NH;
            const T* o1 = sh + (1 * 2 + (1 - p)) * NH;
            const T* o2 = sh + (2 * 2 + (1 - p)) * NH;
            T* w0 = sh + (0 * 2 + p) * NH;
            T* w1 = sh + (1 * 2 + p) * NH;
            T* w2 = sh + (2 * 2 + p) * NH;
#pragma unroll  // the sites of a thread are independent: their latency chains interleave
            for (int h = t; h < NH; h += NT) {
                const Nbr nb = neighbours<L>(h, p, L);
                T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const int mu = d >> 1;
                    const T jj = (d & 1) ? Js[(mu * 2 + (1 - p)) * NH + nb.n[d]] : Js[(mu * 2 + p) * NH + h];
                    const int idx = nb.n[d];
                    Sx = fma(jj, o0[idx], Sx);
                    Sy = fma(jj, o1[idx], Sy);
                    Sz = fma(jj, o2[idx], Sz);
                }
                T sx = w0[h], sy = w1[h], sz = w2[h];
                ld += coolheat_site<T, false>(sx, sy, sz, Sx, Sy, Sz, eps);
                w0[h] = sx;
                w1[h] = sy;
                w2[h] = sz;
                if (step == 1) {
                    const double dx = sx, dy = sy, dz = sz;
                    en_acc += fma(dz, static_cast<double>(Sz),
                                  fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
                }
            }
            lds_barrier();
        }
        // both sums in one pass, each in block_sum's order (valid in thread 0)
        ld = wave_sum(ld);
        en_acc = wave_sum(en_acc);
        if ((t & 63) == 0) {
            red[t >> 6] = ld;
            red[NT / 64 + (t >> 6)] = en_acc;
        }
        lds_barrier();
        double LD = 0.0, H = 0.0;
        if (t == 0) {
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) LD += red[w];
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) H += red[NT / 64 + w];
            H = -H;
        }
        if (t == 0) {  // the decision kernels' formula and updates, from the LDS copies
            const int x = xs, y = ys;
            W[2 * i] = LD;
            cen[x] = H;
            s_cen[x] = H;
            if (isnan(LD)) atomicOr(e.guard, 8);
            const double b1 = s_beta[i], b2 = s_beta[i + 1];
            const double lnA = b1 * s_en[x] + b2 * s_en[y] - b1 * s_cen[y] - b2 * s_cen[x] + LD - s_wh[i];
            st[2 * i] = s_st[2 * i] + 1;
            const bool ok = s_logu[i] < lnA;
            if (ok) {
                s_en[x] = s_cen[x];
                s_en[y] = s_cen[y];
                en[x] = s_en[x];
                en[y] = s_en[y];
                s_sot[i] = y;
                s_sot[i + 1] = x;
                sot[i] = y;
                sot[i + 1] = x;
                tos[x] = i + 1;
                tos[y] = i;
                st[2 * i + 1] = s_st[2 * i + 1] + 1;
            }
            s_ok = ok ? 1 : 0;
        }
        // this wave's requested planes and vectors have landed; the barrier makes every
        // wave's planes visible, and the decision
        __builtin_amdgcn_s_waitcnt(0x0F70);  // gfx9 encoding: vmcnt = 0, expcnt = 7, lgkmcnt = 15
        lds_barrier();
        if (s_ok) {  // uniform: C x over slot xs (it moved to beta_{i+1}), C^-1 y over slot ys
            const size_t gx = static_cast<size_t>(ch) * R + xs;
            const uint4* sv = reinterpret_cast<const uint4*>(sh);
            uint4* xd = reinterpret_cast<uint4*>(spins + gx * 3 * N);
            uint4* yd = reinterpret_cast<uint4*>(spins + gy * 3 * N);
#pragma unroll
            for (int k = 0; k < PC; ++k) {
                const int v = t + k * NT;
                if (v < NV) {
                    xd[v] = sv[v];
                    yd[v] = hv[k];
                }
            }
            lds_barrier();  // the write-back has read the LDS before the next pair cools it
        } else {
            xs = ys;
            cur = 1 - cur;
        }
    }
    // finish the call as coolheat_finish_chain does (every pair attempted: no
    // diagnostics to clear), each slot's round-trip state from its final temperature,
    // the inverse of the labels in LDS, one thread per slot
    __shared__ int s_tos[kChainMaxPairs + 1];
    lds_barrier();
    for (int r = t; r < R; r += NT) s_tos[r] = -1;
    lds_barrier();
    for (int i = t; i < R; i += NT) s_tos[s_sot[i]] = i;
    lds_barrier();
    if (t == 0) e.swap_ctr[ch] += 1u;
    for (int r = t; r < R; r += NT) {
        const int Tr = s_tos[r];
        const size_t k = static_cast<size_t>(ch) * R + r;
        int* rs = e.rt_state + k;
        long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + k;
        if (Tr == 0) {
            if (*rs == 2) *rtt += 1;
            *rs = 1;
        } else if (Tr == R - 1) {
            if (*rs == 1) *rs = 2;
        }
    }
}

template <typename T, int L, int NT, bool PREV, bool HEATALL = false>
static hipError_t go_leg_nt(const hsg_ensemble& e, const ChEps& ce, int i0, int istep, int npc, int blocks,
                            hipStream_t st) {
    constexpr size_t lds = 3 * L * L * L * sizeof(T);
    auto kern = k_coolheat_leg_res<T, L, NT, PREV, HEATALL>;
    const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (a != hipSuccess) return a;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, ce, i0, istep, npc);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t go_leg_res(const hsg_ensemble& e, const ChEps& ce, int i0, int istep, int npc, int blocks, bool prev,
                             hipStream_t st) {
    // one pair per chain: binary32 legs with 1024 threads, binary64 with 512 (its site
    // maps need more than the 128 registers a thread of a 1024-thread workgroup gets)
    constexpr int NH = L * L * L / 2;
    constexpr int NTMAX = sizeof(T) == 4 ? 1024 : 512;
    constexpr int NT1 = NH >= NTMAX ? NTMAX : ((NH + 63) / 64) * 64;
    constexpr int NTS = NT1 > kChThreads ? NT1 : kChThreads;
    if (npc == 1) {
        if (prev) return go_leg_nt<T, L, NTS, true>(e, ce, i0, istep, npc, blocks, st);
        return go_leg_nt<T, L, NTS, false>(e, ce, i0, istep, npc, blocks, st);
    }
    if (prev) return hipErrorInvalidValue;
    // many pairs per launch: binary32 legs with 512 threads, so that the three
    // workgroups one CU's LDS holds at L = 16 carry 24 waves rather than 12 (measured
    // 14 % faster at L = 16; binary64 legs, at 151 registers, lose occupancy instead)
    constexpr int NTM = (sizeof(T) == 4 && NH >= 512) ? 512 : kChThreads;
    return go_leg_nt<T, L, NTM, false>(e, ce, i0, istep, npc, blocks, st);
}

// Legs of the pairs i0 + istep m; prev (ascending, one pair per chain, L <= 16): the
// cooling legs first decide and copy pair i0 - 1.
template <typename T>
static hipError_t go_legs(const hsg_ensemble& e, const ChEps& ce, int i0, int istep, int npc, bool prev,
                          hipStream_t st) {
    const int blocks = e.n_samples * e.n_chains * npc * 2;
    switch (e.L) {
        case 4: return go_leg_res<T, 4>(e, ce, i0, istep, npc, blocks, prev, st);
        case 6: return go_leg_res<T, 6>(e, ce, i0, istep, npc, blocks, prev, st);
        case 8: return go_leg_res<T, 8>(e, ce, i0, istep, npc, blocks, prev, st);
        case 10: return go_leg_res<T, 10>(e, ce, i0, istep, npc, blocks, prev, st);
        case 12: return go_leg_res<T, 12>(e, ce, i0, istep, npc, blocks, prev, st);
        case 14: return go_leg_res<T, 14>(e, ce, i0, istep, npc, blocks, prev, st);
        case 16: return go_leg_res<T, 16>(e, ce, i0, istep, npc, blocks, prev, st);
        default: {
            // one pair per chain: 1024 threads in binary32, 512 in binary64 (as above)
            constexpr int NTG = sizeof(T) == 4 ? 1024 : 512;
            if (npc == 1 && prev)
                hipLaunchKernelGGL((k_coolheat_leg<T, NTG, true>), dim3(blocks), dim3(NTG), 0, st, e, ce, i0, istep,
                                   npc);
            else if (npc == 1)
                hipLaunchKernelGGL((k_coolheat_leg<T, NTG, false>), dim3(blocks), dim3(NTG), 0, st, e, ce, i0, istep,
                                   npc);
            else if (prev)
                return hipErrorInvalidValue;
            else
                hipLaunchKernelGGL((k_coolheat_leg<T, kChThreads, false>), dim3(blocks), dim3(kChThreads), 0, st, e,
                                   ce, i0, istep, npc);
            return hipGetLastError();
        }
    }
}

// istep: 1 for an ascending pass, 2 for an even / odd call with one pair per chain.
static hipError_t launch_decide_copy(const hsg_ensemble& e, int i, int istep, int last, hipStream_t st) {
    const int n_chains = e.n_samples * e.n_chains;
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_coolheat_decide_copy<double>, dim3(n_chains), dim3(kDecideCopyThreads), 0, st, e, i,
                           istep, last);
    else
        hipLaunchKernelGGL(k_coolheat_decide_copy<float>, dim3(n_chains), dim3(kDecideCopyThreads), 0, st, e, i,
                           istep, last);
    return hipGetLastError();
}

static hipError_t coolheat_round(const hsg_ensemble& e, const ChEps& ce, int i0, int istep, int npc, int last,
                                 hipStream_t st) {
    const int n_chains = e.n_samples * e.n_chains;
    hipError_t err = hipSuccess;
    if (npc > 0) {
        err = e.precision == HSG_FP64 ? go_legs<double>(e, ce, i0, istep, npc, false, st)
                                      : go_legs<float>(e, ce, i0, istep, npc, false, st);
        if (err != hipSuccess) return err;
    }
    if (npc == 1) return launch_decide_copy(e, i0, istep, last, st);  // decision and copy-back in one launch
    if (npc == 0) {  // no pair selected (R = 2, odd pairs): the counters alone
        hipLaunchKernelGGL(k_coolheat_finish, dim3((n_chains + 63) / 64), dim3(64), 0, st, e, i0, istep);
        return hipGetLastError();
    }
    (void)last;  // even / odd pairs: one call is one round
    hipLaunchKernelGGL(k_coolheat_decide, dim3((n_chains * npc + 63) / 64), dim3(64), 0, st, e, i0, istep, npc);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int blocks = n_chains * npc * 2;
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_coolheat_copyback<double>, dim3(blocks), dim3(256), 0, st, e, i0, istep, npc);
    else
        hipLaunchKernelGGL(k_coolheat_copyback<float>, dim3(blocks), dim3(256), 0, st, e, i0, istep, npc);
    return hipGetLastError();
}

// ---------------------------------------------------------------- split ascending pass
// For L > 16 with few chains, each leg of pair i is spread over G workgroups, each
// owning a slice of both sublattices, in two launches: k_ch_split_a maps the slice of
// the leg's first sublattice (neighbours and own spins from the source configuration,
// result into the slot's candidate buffer) and copies the slice of the other
// sublattice; k_ch_split_b maps the second sublattice in the candidate buffer.  Each
// leaves per-slice sums (log Jacobian, energy).  The decision of pair i is taken by
// the cooling workgroups of pair i + 1 (every one alike, from the sums) before they
// start, as only that leg depends on it; one of them updates the labels, counters and
// energies, and each copies its slice of the accepted candidates over their spins.
// The last pair is decided by k_ch_split_decide, and k_ch_split_finish advances the
// exchange counter and the round trips.  Per chain and pair parity (pair i's sums are
// written while pair i - 1's are read), in the scratch's partial area: ld[2][G],
// h[2][G] and a record of both legs' slots and energies before the pair.  A slice is
// the same range of sites h in every sublattice and component, for the maps and the
// copies alike, so each site is copied and mapped by the workgroup that owns it.
struct ChSplit {
    double* ld;   // [leg][G] log Jacobian per slice (both half-steps)
    double* hs;   // [leg][G] energy sum per slice (second half-step)
    double* en;   // [leg] energy of the leg's configuration before the pair
    int* slot;    // [leg] the leg's slot
};

__device__ __forceinline__ ChSplit ch_split(const hsg_ensemble& e, int ch, int G, int i) {
    const ScratchLayout sl = scratch_layout(e);
    double* base = reinterpret_cast<double*>(static_cast<unsigned char*>(e.scratch) + sl.partial) +
                   (static_cast<size_t>(ch) * 2 + (i & 1)) * (4 * G + 3);
    ChSplit c;
    c.ld = base;
    c.hs = base + 2 * G;
    c.en = base + 4 * G;
    c.slot = reinterpret_cast<int*>(base + 4 * G + 2);
    return c;
}

// Pair i's acceptance from the records and sums (read-only while it is evaluated):
// ln A = b1 H(x) + b2 H(y) - b1 H(C^-1 y) - b2 H(C x) + ln det J(x) - ln det J(C^-1 y).
struct ChDecision {
    bool ok;
    int x, y;
    double ld0, ld1, hx, hy;
};

__device__ __forceinline__ ChDecision ch_split_decision(const hsg_ensemble& e, int ch, int i, int G,
                                                        const ChSplit& c) {
    ChDecision d;
    d.x = c.slot[0];
    d.y = c.slot[1];
    d.ld0 = d.ld1 = d.hx = d.hy = 0.0;
    for (int g = 0; g < G; ++g) {
        d.ld0 += c.ld[g];
        d.ld1 += c.ld[G + g];
        d.hx += c.hs[g];
        d.hy += c.hs[G + g];
    }
    d.hx = -d.hx;  // H(C x) and H(C^-1 y)
    d.hy = -d.hy;
    const double b1 = e.betas[i], b2 = e.betas[i + 1];
    const double lnA = b1 * c.en[0] + b2 * c.en[1] - b1 * d.hy - b2 * d.hx + d.ld0 - d.ld1;
    const Words w = philox(static_cast<uint32_t>(i), e.swap_ctr[ch], e.chain_base + static_cast<uint32_t>(ch),
                           kTagSwap << 24, key_lo(e.seed), key_hi(e.seed));
    d.ok = log(u01_52(w.w0, w.w1)) < lnA;
    return d;
}

// Labels, counters, energies and diagnostics of pair i after its decision (one thread).
__device__ __forceinline__ void ch_split_commit(const hsg_ensemble& e, int ch, int i, const ChDecision& d) {
    const int R = e.n_temps;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    double* W = e.work + static_cast<size_t>(ch) * (R - 1) * 2;
    W[2 * i] = d.ld0;
    W[2 * i + 1] = d.ld1;
    if (isnan(d.ld0) || isnan(d.ld1)) atomicOr(e.guard, 8);
    st[2 * i] += 1;
    if (d.ok) {
        int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
        int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
        double* en = e.energy + static_cast<size_t>(ch) * R;
        en[d.x] = d.hx;
        en[d.y] = d.hy;
        sot[i] = d.y;
        sot[i + 1] = d.x;
        tos[d.x] = i + 1;
        tos[d.y] = i;
        st[2 * i + 1] += 1;
    }
}

// Slice [h0, h1) of every sublattice and component of candidate `slot` over its spins.
template <typename T>
__device__ __forceinline__ void ch_split_copy(const hsg_ensemble& e, size_t slot, int N, int h0, int h1) {
    const ScratchLayout sl = scratch_layout(e);
    const int NH = N / 2;
    const T* src = reinterpret_cast<const T*>(static_cast<unsigned char*>(e.scratch) + sl.cand) + slot * 3 * N;
    T* dst = static_cast<T*>(e.spins) + slot * 3 * N;
    for (int plane = 0; plane < 6; ++plane)
        for (int h = h0 + static_cast<int>(threadIdx.x); h < h1; h += kChThreads)
            dst[plane * NH + h] = src[plane * NH + h];
}

// One half-step of a leg over sites [h0, h1) of sublattice p: fields from `nbr`, own
// spins from `own`, results into `out` (may equal `own`); returns the log Jacobians'
// sum and adds s'.S to *en if `want`.
template <typename T, bool HEAT>
__device__ __forceinline__ double ch_split_half(const T* nbr, const T* own, T* out, const T* __restrict__ J, int L,
                                                int p, int h0, int h1, T eps, bool want, double* en) {
    const int NH = L * L * L / 2;
    const T* o0 = nbr + (0 * 2 + (1 - p)) * NH;
    const T* o1 = nbr + (1 * 2 + (1 - p)) * NH;
    const T* o2 = nbr + (2 * 2 + (1 - p)) * NH;
    double ld = 0.0;
    for (int h = h0 + static_cast<int>(threadIdx.x); h < h1; h += kChThreads) {
        const Nbr nb = neighbours<0>(h, p, L);
        T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const int mu = d >> 1;
            const T jj = (d & 1) ? J[(mu * 2 + (1 - p)) * NH + nb.n[d]] : J[(mu * 2 + p) * NH + h];
            const int idx = nb.n[d];
            Sx = fma(jj, o0[idx], Sx);
            Sy = fma(jj, o1[idx], Sy);
            Sz = fma(jj, o2[idx], Sz);
        }
        T sx = own[(0 * 2 + p) * NH + h], sy = own[(1 * 2 + p) * NH + h], sz = own[(2 * 2 + p) * NH + h];
        ld += coolheat_site<T, HEAT>(sx, sy, sz, Sx, Sy, Sz, eps);
        out[(0 * 2 + p) * NH + h] = sx;
        out[(1 * 2 + p) * NH + h] = sy;
        out[(2 * 2 + p) * NH + h] = sz;
        if (want) {
            const double dx = sx, dy = sy, dz = sz;
            *en += fma(dz, static_cast<double>(Sz), fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
        }
    }
    return ld;
}

// Workgroup (chain, leg, slice g) of pair i's first launch.
template <typename T>
__global__ void __launch_bounds__(kChThreads) k_ch_split_a(hsg_ensemble e, ChEps ce, int i, int G) {
    __shared__ double red[kChThreads / 64];
    const T eps = ch_eps<T>(ce, i);
    const int L = e.L, N = L * L * L, NH = N / 2, R = e.n_temps;
    const int b = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));  // a chain's slices on one XCD
    const int g = b % G, leg = (b / G) & 1, ch = b / (2 * G);
    const ChSplit c = ch_split(e, ch, G, i);
    const ScratchLayout sl = scratch_layout(e);
    T* cand = reinterpret_cast<T*>(static_cast<unsigned char*>(e.scratch) + sl.cand);
    T* spins = static_cast<T*>(e.spins);
    const int h0 = static_cast<int>(static_cast<long long>(NH) * g / G);
    const int h1 = static_cast<int>(static_cast<long long>(NH) * (g + 1) / G);
    int slot;
    double en_before;
    bool from_cand = false;
    if (leg == 0 && i > 0) {  // decide pair i - 1 first (uniform over the workgroup)
        const ChSplit cp = ch_split(e, ch, G, i - 1);
        const ChDecision d = ch_split_decision(e, ch, i - 1, G, cp);
        if (d.ok) {  // its candidates become the spins of their slots, this slice here
            ch_split_copy<T>(e, static_cast<size_t>(ch) * R + d.x, N, h0, h1);
            ch_split_copy<T>(e, static_cast<size_t>(ch) * R + d.y, N, h0, h1);
            __syncthreads();  // C x of this slice is saved before the map overwrites it
        }
        slot = d.ok ? d.x : cp.slot[1];
        en_before = d.ok ? d.hx : cp.en[1];
        from_cand = d.ok;
        if (g == 0 && threadIdx.x == 0) ch_split_commit(e, ch, i - 1, d);
    } else {
        slot = label(e.slot_of_temp[ch * R + i + leg], R, e.guard);
        en_before = e.energy[static_cast<size_t>(ch) * R + slot];
    }
    const size_t gs = static_cast<size_t>(ch) * R + slot;
    const T* src = (from_cand ? cand : spins) + gs * 3 * N;
    T* dst = cand + gs * 3 * N;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(ch / e.n_chains) * 3 * N;
    const int p = leg;  // cooling maps sublattice 0 first, heating sublattice 1
    double unused = 0.0;
    const double ld = leg ? ch_split_half<T, true>(src, src, dst, J, L, p, h0, h1, eps, false, &unused)
                          : ch_split_half<T, false>(src, src, dst, J, L, p, h0, h1, eps, false, &unused);
    if (!from_cand) {  // the slice of the other sublattice into the candidate buffer
        const int q = 1 - p;
        for (int mu = 0; mu < 3; ++mu)
            for (int h = h0 + static_cast<int>(threadIdx.x); h < h1; h += kChThreads)
                dst[(mu * 2 + q) * NH + h] = src[(mu * 2 + q) * NH + h];
    }
    const double LD = block_sum<kChThreads>(ld, red);
    if (threadIdx.x == 0) {
        c.ld[leg * G + g] = LD;
        if (g == 0) {
            c.slot[leg] = slot;
            c.en[leg] = en_before;
        }
    }
}

// Workgroup (chain, leg, slice g) of pair i's second launch.
template <typename T>
__global__ void __launch_bounds__(kChThreads) k_ch_split_b(hsg_ensemble e, ChEps ce, int i, int G) {
    __shared__ double red[kChThreads / 64];
    const T eps = ch_eps<T>(ce, i);
    const int L = e.L, N = L * L * L, NH = N / 2, R = e.n_temps;
    const int b = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));  // a chain's slices on one XCD
    const int g = b % G, leg = (b / G) & 1, ch = b / (2 * G);
    const ChSplit c = ch_split(e, ch, G, i);
    const ScratchLayout sl = scratch_layout(e);
    T* dst = reinterpret_cast<T*>(static_cast<unsigned char*>(e.scratch) + sl.cand) +
             (static_cast<size_t>(ch) * R + c.slot[leg]) * 3 * N;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(ch / e.n_chains) * 3 * N;
    const int p = 1 - leg;
    const int h0 = static_cast<int>(static_cast<long long>(NH) * g / G);
    const int h1 = static_cast<int>(static_cast<long long>(NH) * (g + 1) / G);
    double en = 0.0;
    const double ld = leg ? ch_split_half<T, true>(dst, dst, dst, J, L, p, h0, h1, eps, true, &en)
                          : ch_split_half<T, false>(dst, dst, dst, J, L, p, h0, h1, eps, true, &en);
    const double LD = block_sum<kChThreads>(ld, red);
    const double EN = block_sum<kChThreads>(en, red);
    if (threadIdx.x == 0) {
        c.ld[leg * G + g] += LD;
        c.hs[leg * G + g] = EN;
    }
}

// The last pair: decision, slice-wise copy of accepted candidates, commit.
template <typename T>
__global__ void __launch_bounds__(kChThreads) k_ch_split_decide(hsg_ensemble e, int i, int G) {
    const int N = e.L * e.L * e.L, R = e.n_temps;
    const int b = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));  // a chain's slices on one XCD
    const int g = b % G, ch = b / G;
    const ChSplit c = ch_split(e, ch, G, i);
    const ChDecision d = ch_split_decision(e, ch, i, G, c);
    if (d.ok) {
        const int NH = N / 2;
        const int h0 = static_cast<int>(static_cast<long long>(NH) * g / G);
        const int h1 = static_cast<int>(static_cast<long long>(NH) * (g + 1) / G);
        ch_split_copy<T>(e, static_cast<size_t>(ch) * R + d.x, N, h0, h1);
        ch_split_copy<T>(e, static_cast<size_t>(ch) * R + d.y, N, h0, h1);
    }
    if (g == 0 && threadIdx.x == 0) ch_split_commit(e, ch, i, d);
}

// Per chain, after the pass: exchange counter and round trips.
__global__ void k_ch_split_finish(hsg_ensemble e) {
    // one thread per (chain, slot): slot r's round-trip state from its temperature; the
    // thread of slot 0 advances the chain's counter
    const int n_chains = e.n_samples * e.n_chains;
    const int R = e.n_temps;
    const long long b = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= static_cast<long long>(n_chains) * R) return;
    const int ch = static_cast<int>(b / R), r = static_cast<int>(b % R);
    if (r == 0) e.swap_ctr[ch] += 1u;
    const size_t k = static_cast<size_t>(ch) * R + r;
    const int Tr = e.temp_of_slot[k];
    int* rs = e.rt_state + k;
    long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + k;
    if (Tr == 0) {
        if (*rs == 2) *rtt += 1;
        *rs = 1;
    } else if (Tr == R - 1) {
        if (*rs == 1) *rs = 2;
    }
}

// Workgroups per leg for the split pass (L > 16): about 512 workgroups per launch, at
// least 512 sites per slice, within the scratch's partial area; 1 = not split.
static int ch_split_groups(const hsg_ensemble& e) {
    if (e.L <= 16) return 1;
    const int chains = e.n_samples * e.n_chains;
    const long long NH = static_cast<long long>(e.L) * e.L * e.L / 2;
    const ScratchLayout sl = scratch_layout(e);
    const long long per_chain = static_cast<long long>(e.n_temps) * sl.max_tiles;  // doubles
    long long G = (256 + chains - 1) / chains;
    G = G < NH / 512 ? G : NH / 512;
    G = G < (per_chain / 2 - 3) / 4 ? G : (per_chain / 2 - 3) / 4;  // two pair parities
    return G < 2 ? 1 : static_cast<int>(G);
}

template <typename T>
static hipError_t coolheat_split_pass(const hsg_ensemble& e, const ChEps& ce, int G, hipStream_t st) {
    const int chains = e.n_samples * e.n_chains, R = e.n_temps;
    for (int i = 0; i < R - 1; ++i) {
        hipLaunchKernelGGL(k_ch_split_a<T>, dim3(chains * 2 * G), dim3(kChThreads), 0, st, e, ce, i, G);
        hipLaunchKernelGGL(k_ch_split_b<T>, dim3(chains * 2 * G), dim3(kChThreads), 0, st, e, ce, i, G);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_ch_split_decide<T>, dim3(chains * G), dim3(kChThreads), 0, st, e, R - 2, G);
    const long long n_fin = static_cast<long long>(chains) * R;
    hipLaunchKernelGGL(k_ch_split_finish, dim3(static_cast<unsigned>((n_fin + 255) / 256)), dim3(256), 0, st, e);
    return hipGetLastError();
}

// Ascending binary32 pass at L <= 16 in two launches: every pair's heating leg at once,
// then one workgroup per chain for the cooling legs and decisions (thread counts as in
// the per-pair launches, so the sums are the same).  hipErrorNotSupported if the
// couplings and two replicas do not fit one workgroup's LDS.
template <int L>
static hipError_t coolheat_asc_two_L(const hsg_ensemble& e, const ChEps& ce, hipStream_t st) {
    constexpr int NH = L * L * L / 2;
    constexpr int NT1 = NH >= 1024 ? 1024 : ((NH + 63) / 64) * 64;
    constexpr int NTS = NT1 > kChThreads ? NT1 : kChThreads;
    constexpr size_t lds = 3 * 3 * L * L * L * sizeof(float);
    const int chains = e.n_samples * e.n_chains, R = e.n_temps;
    if (lds > max_block_lds() || R - 1 > kChainMaxPairs) return hipErrorNotSupported;
    hipError_t err = go_leg_nt<float, L, NTS, false, true>(e, ce, 0, 1, 1, chains * (R - 1), st);
    if (err != hipSuccess) return err;
    auto kern = k_coolheat_cool_chain<L, NTS>;
    err = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(chains), dim3(NTS), lds, st, e, ce);
    return hipGetLastError();
}

static hipError_t coolheat_asc_two(const hsg_ensemble& e, const ChEps& ce, hipStream_t st) {
    switch (e.L) {
        case 4: return coolheat_asc_two_L<4>(e, ce, st);
        case 6: return coolheat_asc_two_L<6>(e, ce, st);
        case 8: return coolheat_asc_two_L<8>(e, ce, st);
        case 10: return coolheat_asc_two_L<10>(e, ce, st);
        case 12: return coolheat_asc_two_L<12>(e, ce, st);
        case 14: return coolheat_asc_two_L<14>(e, ce, st);
        case 16: return coolheat_asc_two_L<16>(e, ce, st);
        default: return hipErrorNotSupported;
    }
}

hipError_t launch_coolheat(const hsg_ensemble& e, int pairing, double eps, const double* eps_pair, hipStream_t st) {
    const ChEps ce{eps, eps_pair};
    const int R = e.n_temps;
    if (e.n_samples * e.n_chains <= 0 || R < 2) return hipSuccess;
    if (pairing == 0) {
        // ascending order: each pair sees the states the previous pair left
        const int G = ch_split_groups(e);
        if (G > 1)
            return e.precision == HSG_FP64 ? coolheat_split_pass<double>(e, ce, G, st)
                                           : coolheat_split_pass<float>(e, ce, G, st);
        if (e.precision == HSG_FP32 && e.L <= 16) {
            const hipError_t err = coolheat_asc_two(e, ce, st);
            if (err != hipErrorNotSupported) return err;
        }
        // (pair i - 1 decided inside pair i's launch, the last pair by its own)
        for (int i = 0; i < R - 1; ++i) {
            hipError_t err = e.precision == HSG_FP64 ? go_legs<double>(e, ce, i, 1, 1, i > 0, st)
                                                     : go_legs<float>(e, ce, i, 1, 1, i > 0, st);
            if (err != hipSuccess) return err;
        }
        return launch_decide_copy(e, R - 2, 1, 1, st);
    }
    const int first = pairing == 1 ? 0 : 1;
    const int npc = (R - first) / 2;
    return coolheat_round(e, ce, first, 2, npc, 1, st);
}

}  // namespace hsg
