// Device code of the LDS-resident sweeps, shared by their kernels (sweep_resident.hip)
// and the persistent batch kernel (sweep_batch.hip).
//
// One workgroup owns one replica: its whole lattice [3][2][N/2] sits in LDS for
// every half-sweep of the launch (n sweeps of a regular step, or the K sweeps
// of an annealing leg), so HBM sees one read and one write of the replica per
// launch.  Each thread owns fixed site pairs (h, h + N/4) of both sublattices
// and keeps their six couplings in registers (neighbour offsets are recomputed).  Sites
// of one sublattice never interact (paper Sec. III.A), so a half-sweep is one
// barrier-separated LDS pass; the energy H = -sum_{x in p} s_x.S_x is fused
// into the last half-sweep of each sweep (every bond has one end in p).
#pragma once

#include "hsg_device.h"

namespace hsg {

template <typename T, int MQ>
struct Owned {
    T j[2][MQ][2][6];  // [parity][pair][half][direction] couplings of the owned sites
};

// Owned-site geometry.  Thread t owns the sites h = q_m + NQ half of each
// sublattice (h = ih + (L/2)(j + L k), x = 2 ih + o, o = (p + j + k) & 1), m < MQ;
// q_m is also the site's Philox counter, shared by its two halves.  In general
// q_m = t + NT m.  When NT is a whole number G of sublattice k-planes (L/2 * L
// sites), NT divides NQ and the owned planes of a thread keep the parity of k,
// all sites of a thread share (ih, j, o): their neighbours are those of the first
// site shifted by compile-time offsets, except the z-neighbours across the
// periodic boundary, which only the first site (-z) and the last site (+z) can
// have.  Nine per-thread indices then address every neighbour and the site
// offsets fold into the LDS instructions.  With G even and MQ >= 2 (z-pairs), a
// thread owns the planes k0 + 2m of each half, k0 = (g & 1) + 2 MQ (g >> 1) for
// the thread's plane group g = t / (L/2 * L): the +z neighbour of its site m is
// the -z neighbour of its site m + 1, read once (MQ + 1 instead of 2 MQ z-reads
// per half); otherwise the planes g + G m (G even, or MQ = 1).
template <int L, int NT>
struct SiteMap {
    static constexpr int HL = L / 2, N = L * L * L, NQ = N / 4, PLANE = HL * L;
    static constexpr int MQ = (NQ + NT - 1) / NT;
    static constexpr int STEPK = NT / PLANE;
    static constexpr bool invariant = (NT % PLANE == 0) && (NQ % NT == 0) &&
                                      (STEPK % 2 == 0 || MQ == 1) && ((L / 2) % 2 == 0);
    static constexpr bool zpair = invariant && (STEPK % 2 == 0) && MQ >= 2;
    static constexpr int STEPM = zpair ? 2 * PLANE : NT;  // site offset between m and m + 1
};

// Counter (site index within the first half) of owned site m of thread t.
template <int L, int NT>
__device__ __forceinline__ int owned_q(int t, int m) {
    using M = SiteMap<L, NT>;
    if constexpr (M::zpair) {
        const int g = t / M::PLANE;
        return t - g * M::PLANE + M::PLANE * ((g & 1) + 2 * M::MQ * (g >> 1)) + M::STEPM * m;
    } else {
        return t + NT * m;
    }
}

struct FirstNbr {
    int x[2][2];  // [parity][+x, -x] of the first site
    int yp, ym;   // +y, -y of the first site (either parity)
    int zm_first, zp_last;
    int q0;       // the first site
};

template <int L, int NT>
__device__ __forceinline__ FirstNbr first_neighbours(int t) {
    using M = SiteMap<L, NT>;
    FirstNbr f;
    const int q0 = M::invariant ? owned_q<L, NT>(t, 0) : t;
    const Nbr a = neighbours<L>(q0, 0, L), b = neighbours<L>(q0, 1, L);
    f.x[0][0] = a.n[0];
    f.x[0][1] = a.n[1];
    f.x[1][0] = b.n[0];
    f.x[1][1] = b.n[1];
    f.yp = a.n[2];
    f.ym = a.n[3];
    f.zm_first = a.n[5];
    f.zp_last = neighbours<L>(q0 + M::STEPM * (M::MQ - 1) + M::NQ, 0, L).n[4];
    f.q0 = q0;
    return f;
}

// Vector v of a replica as loaded into LDS: all six planes in order, or
// (parity1_only) the three parity-1 planes, plane mu at (2 mu + 1) NVP.
template <int NVP>
__device__ __forceinline__ int loaded_vec(int v, bool parity1_only) {
    if (!parity1_only) return v;
    const int mu = v / NVP;
    return (2 * mu + 1) * NVP + (v - mu * NVP);
}

// Neighbours of owned site (m, half) of parity p, h = t + NT m + NQ half.
template <int L, int NT, int MQ>
__device__ __forceinline__ Nbr site_nbrs(const FirstNbr& fn, int p, int m, int half, int h, int t) {
    using M = SiteMap<L, NT>;
    Nbr nb;
    if constexpr (M::invariant) {
        const int c = M::STEPM * m + M::NQ * half;
        nb.n[0] = fn.x[p][0] + c;
        nb.n[1] = fn.x[p][1] + c;
        nb.n[2] = fn.yp + c;
        nb.n[3] = fn.ym + c;
        nb.n[4] = (m == MQ - 1 && half == 1) ? fn.zp_last : fn.q0 + M::PLANE + c;
        nb.n[5] = (m == 0 && half == 0) ? fn.zm_first : fn.q0 - M::PLANE + c;
    } else {
        nb = neighbours<L>(h, p, L);
    }
    return nb;
}

// The six couplings of every owned site, from a coupling array [3][2][NH] (global
// memory or its LDS copy): the bond to +mu is stored at the site, the bond to -mu
// at the -mu neighbour.
template <typename T, int L, int NT, int MQ>
__device__ __forceinline__ void load_owned(Owned<T, MQ>& own, const T* __restrict__ J,
                                           const FirstNbr& fn, int t) {
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int m = 0; m < MQ; ++m)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int q = SiteMap<L, NT>::invariant ? owned_q<L, NT>(t, m) : t + NT * m;
                const int h = (q < NQ ? q : 0) + half * NQ;
                const Nbr nb = site_nbrs<L, NT, MQ>(fn, p, m, half, h, t);
#pragma unroll
                for (int mu = 0; mu < 3; ++mu) {
                    own.j[p][m][half][2 * mu] = J[(mu * 2 + p) * NH + h];
                    own.j[p][m][half][2 * mu + 1] = J[(mu * 2 + (1 - p)) * NH + nb.n[2 * mu + 1]];
                }
            }
}

// One half-sweep over the sites of parity P (compile-time), HB or OR.  KIND 0 takes
// the kind, the renormalisation and the energy from the arguments; KIND 1 (heat-bath)
// and 2 (overrelaxation) fix them at compile time, without renormalisation or energy,
// so that the owned sites form one branch-free block the compiler can schedule as a
// whole (the LDS reads of a site issued under the arithmetic of the one before).
template <typename T, int L, int NT, int MQ, int P, int KIND = 0>
__device__ __forceinline__ void resident_half(T* __restrict__ sh, const Owned<T, MQ>& own,
                                              const FirstNbr& fn, bool hb_arg, bool rn_arg, int hs, T beta,
                                              uint32_t tsw, uint32_t g, uint32_t k0, uint32_t k1,
                                              bool want_arg, double& acc, bool& bad, int t) {
    const bool hb = KIND == 0 ? hb_arg : KIND == 1;
    const bool rn = KIND == 0 && rn_arg;
    const bool want = KIND == 0 && want_arg;
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
    constexpr bool INV = SiteMap<L, NT>::invariant;
    const T* __restrict__ o0 = sh + (0 * 2 + (1 - P)) * NH;
    const T* __restrict__ o1 = sh + (1 * 2 + (1 - P)) * NH;
    const T* __restrict__ o2 = sh + (2 * 2 + (1 - P)) * NH;
    T* __restrict__ w0 = sh + (0 * 2 + P) * NH;
    T* __restrict__ w1 = sh + (1 * 2 + P) * NH;
    T* __restrict__ w2 = sh + (2 * 2 + P) * NH;
    constexpr bool ZP = SiteMap<L, NT>::zpair;
    const uint32_t c3 = heatbath_c3(hs);
    T zc[2][3];  // z-pairs: the +z neighbour of site (m - 1, half), the -z one of (m, half)
#pragma unroll
    for (int m = 0; m < MQ; ++m) {
        int q = INV ? fn.q0 + SiteMap<L, NT>::STEPM * m : t + NT * m;
        // Generic geometry: an opaque copy keeps the site arithmetic (neighbour
        // offsets, LDS addresses) inside each half-sweep instead of letting it be
        // hoisted and held live in registers across the whole kernel (empty asm,
        // no instruction emitted).
        if (!INV) asm volatile("" : "+v"(q));
        if ((NQ % NT) != 0 && q >= NQ) break;
        Words wq{0, 0, 0, 0};
        if (sizeof(T) == 4 && hb) wq = philox(static_cast<uint32_t>(q), tsw, g, c3, k0, k1);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int h = q + half * NQ;
            const Nbr nb = site_nbrs<L, NT, MQ>(fn, P, m, half, h, t);
            T Sx = T(0), Sy = T(0), Sz = T(0);
            T zm[3];  // the -z neighbour carried from site (m - 1, half)
            if (ZP && m > 0) {
                zm[0] = zc[half][0];
                zm[1] = zc[half][1];
                zm[2] = zc[half][2];
            }
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int idx = nb.n[d];
                const T jj = own.j[P][m][half][d];
                T vx, vy, vz;
                if (ZP && d == 5 && m > 0) {
                    vx = zm[0];
                    vy = zm[1];
                    vz = zm[2];
                } else {
                    vx = o0[idx];
                    vy = o1[idx];
                    vz = o2[idx];
                }
                if (ZP && d == 4) {
                    zc[half][0] = vx;
                    zc[half][1] = vy;
                    zc[half][2] = vz;
                }
                Sx = fma(jj, vx, Sx);
                Sy = fma(jj, vy, Sy);
                Sz = fma(jj, vz, Sz);
            }
            T ox, oy, oz;
            if (hb) {
                T r1, r2;
                if (sizeof(T) == 4) {
                    r1 = static_cast<T>(u01_23(half ? wq.w2 : wq.w0));
                    r2 = static_cast<T>(u01_23(half ? wq.w3 : wq.w1));
                } else {
                    const Words wd = philox(static_cast<uint32_t>(h), tsw, g, c3, k0, k1);
                    r1 = static_cast<T>(u01_52(wd.w0, wd.w1));
                    r2 = static_cast<T>(u01_52(wd.w2, wd.w3));
                }
                heatbath<T>(Sx, Sy, Sz, beta, r1, r2, ox, oy, oz);
            } else {
                overrelax<T>(w0[h], w1[h], w2[h], Sx, Sy, Sz, ox, oy, oz);
                if (rn) renormalize(ox, oy, oz);
            }
            w0[h] = ox;
            w1[h] = oy;
            w2[h] = oz;
            if (want) {
                const double dx = ox, dy = oy, dz = oz;
                acc += fma(dz, static_cast<double>(Sz),
                           fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
                const double n2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (!(fabs(n2 - 1.0) <= NormTol<T>::value)) bad = true;
            }
        }
    }
}

// Work item of a workgroup: xcd_order(blockIdx.x) (consecutive work items, which
// share a sample and its couplings, run on one XCD).
// mode 0: regular sweeps of slot (work item) at its own temperature.
// mode 1: annealing legs of the pairs with i mod 2 == parity; block ->
//         (chain, pair, leg); leg 0 = up (forward order), 1 = down (adjoint).
// The work of one workgroup: work item `bid` (see above), the replica in the LDS at
// smem_raw, `red` and `s_H` workgroup-shared scratch of >= NT/64 and 1 doubles.  Used
// by k_resident and by the persistent batch kernel (sweep_batch.hip).  KEEP (regular
// sweeps of replicas of one sample in a row): 1 loads the couplings into *keep, 2 takes
// them from there and loads only the replica.  FIXED_KINDS: bit 0 runs heat-bath, bit 1
// overrelaxation half-sweeps (without renormalisation or energy) in the form with the
// kind fixed at compile time, the others in the general form.
template <typename T, int L, int NT, int KEEP = 0, int FIXED_KINDS = 3>
__device__ __forceinline__ void resident_item(const hsg_ensemble& e, int bid, int n_sweeps, int n_hb, int n_or,
                                              int anneal, int parity, unsigned char* smem_raw, double* red,
                                              double& s_H,
                                              Owned<T, (L * L * L / 4 + NT - 1) / NT>* keep = nullptr) {
    const int tid = static_cast<int>(threadIdx.x);
    constexpr int N = L * L * L, NQ = N / 4;
    constexpr int MQ = (NQ + NT - 1) / NT;
    T* sh = reinterpret_cast<T*>(smem_raw);

    const int C = e.n_chains, R = e.n_temps;
    int slot, leg = 0, ipair = 0, K = n_sweeps, ch = 0;
    double lam_a = 0.0, lam_b = 0.0;
    const double* lam_tab = nullptr;
    if (!anneal) {
        slot = bid;
    } else {
        const int npp = (R - parity) / 2;
        leg = bid & 1;
        const int rest = bid >> 1;
        ch = rest / npp;
        ipair = parity + 2 * (rest % npp);
        slot = ch * R + label(e.slot_of_temp[ch * R + ipair + leg], R, e.guard);
        K = e.anneal_K[ipair];
        if (K < 0 || K > e.anneal_K_max) {
            if (tid == 0) atomicOr(e.guard, 2);
            K = K < 0 ? 0 : e.anneal_K_max;
        }
        lam_a = e.betas[ipair];
        lam_b = e.betas[ipair + 1];
        if (e.anneal_lambda) lam_tab = e.anneal_lambda + static_cast<size_t>(ipair) * e.anneal_K_max;
    }
    const int smp = slot / (C * R);
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* gs = static_cast<T*>(e.spins) + static_cast<size_t>(slot) * 3 * N;
    const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
    const uint32_t t0 = e.sweep_ctr[slot];
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);

    // protocol point k of this leg (k = 0 .. K+1), ascending for the up-leg
    auto lam = [&](int k) -> double {
        if (k <= 0) return lam_a;
        if (k >= K + 1) return lam_b;
        return lam_tab ? lam_tab[k - 1] : lam_a + static_cast<double>(k) * (lam_b - lam_a) / static_cast<double>(K + 1);
    };

    double H = anneal ? e.energy[slot] : 0.0;
    if (anneal && K == 0) {
        if (tid == 0) {
            const double W = leg == 0 ? (lam_b - lam_a) * H : (lam_a - lam_b) * H;
            e.work[(static_cast<size_t>(ch) * (R - 1) + ipair) * 2 + leg] = W;
            reinterpret_cast<double*>(scr + sl.cand_energy)[slot] = H;
        }
        return;
    }

    // Couplings: global -> LDS (16-byte vectors) -> registers; then the replica ->
    // LDS.  A sweep that opens with a heat-bath half-sweep of parity 0 (every
    // regular sweep and forward leg with n_hb > 0) overwrites each parity-0 spin
    // without reading it, as the heat-bath draw depends on the neighbours only:
    // then only the three parity-1 planes are loaded.  Where the vectors fit in
    // registers, the replica's loads are issued right after the couplings' loads
    // and stay in flight while the couplings pass through LDS.
    Owned<T, MQ> own_local;
    Owned<T, MQ>& own = KEEP ? *keep : own_local;
    const FirstNbr fn = first_neighbours<L, NT>(tid);
    if constexpr (KEEP == 2) {  // the couplings are in registers already: the replica only
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
        constexpr int NVP = NV / 6;
        const bool hb_first = n_hb > 0 && n_sweeps > 0;
        const uint4* src = reinterpret_cast<const uint4*>(gs);
        uint4* dst = reinterpret_cast<uint4*>(sh);
        const int n_load = hb_first ? NV / 2 : NV;
        for (int v = tid; v < n_load; v += NT) {
            const int o = loaded_vec<NVP>(v, hb_first);
            dst[o] = src[o];
        }
    } else {
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;  // vectors per replica
        constexpr int NVP = NV / 6;                                    // per plane
        constexpr int PV = (NV + NT - 1) / NT;                         // per thread
        constexpr bool PREFETCH = PV <= 6;
        const bool hb_first = n_hb > 0 && (anneal ? leg == 0 : n_sweeps > 0);
        const uint4* js = reinterpret_cast<const uint4*>(J);
        const uint4* src = reinterpret_cast<const uint4*>(gs);
        uint4* dst = reinterpret_cast<uint4*>(sh);
        const int n_load = hb_first ? NV / 2 : NV;
        if constexpr (PREFETCH) {
            uint4 jv[PV], sv[PV];
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = tid + k * NT;
                jv[k] = (v < NV) ? js[v] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = tid + k * NT;
                sv[k] = (v < n_load) ? src[loaded_vec<NVP>(v, hb_first)] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = tid + k * NT;
                if (v < NV) dst[v] = jv[k];
            }
            lds_barrier();
            load_owned<T, L, NT, MQ>(own, sh, fn, tid);
            lds_barrier();  // every thread holds its couplings before the LDS is reused
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = tid + k * NT;
                if (v < n_load) {
                    const int o = loaded_vec<NVP>(v, hb_first);
                    dst[o] = sv[k];
                }
            }
        } else {
            for (int v = tid; v < NV; v += NT) dst[v] = js[v];
            __syncthreads();
            load_owned<T, L, NT, MQ>(own, sh, fn, tid);
            __syncthreads();
            for (int v = tid; v < n_load; v += NT) {
                const int o = loaded_vec<NVP>(v, hb_first);
                dst[o] = src[o];
            }
        }
    }
    __syncthreads();

    const int nhalf = 2 * (n_hb + n_or);
    const bool adj = anneal && leg == 1;
    const int n_iter = anneal ? K + 1 : n_sweeps;
    double W = 0.0;
    bool bad = false;
    for (int k = 0; k < n_iter; ++k) {
        double beta_d;
        if (anneal) {
            const double cur = adj ? lam(K + 1 - k) : lam(k);
            const double nxt = adj ? lam(K - k) : lam(k + 1);
            W += (nxt - cur) * H;
            if (k == K) break;
            beta_d = nxt;
        } else {
            beta_d = e.betas[label(e.temp_of_slot[slot], R, e.guard)];
        }
        const T beta = static_cast<T>(beta_d);
        const bool need_e = anneal || (k == n_sweeps - 1);
        const uint32_t tsw = t0 + static_cast<uint32_t>(k);
        double acc = 0.0;
        for (int step = 0; step < nhalf; ++step) {
            const int pos = adj ? nhalf - 1 - step : step;  // position in the forward order
            const bool hb = pos < 2 * n_hb;
            const bool rn = renorm_on(e) && n_hb == 0 && pos >= nhalf - 2;  // renormalised once per sweep
            const int p = pos & 1;
            const bool want = need_e && (step == nhalf - 1);
            if (rn || want || !(FIXED_KINDS & (hb ? 1 : 2))) {
                if (p == 0)
                    resident_half<T, L, NT, MQ, 0>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
                else
                    resident_half<T, L, NT, MQ, 1>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
            } else if (hb) {
                if (p == 0)
                    resident_half<T, L, NT, MQ, 0, 1>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
                else
                    resident_half<T, L, NT, MQ, 1, 1>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
            } else {
                if (p == 0)
                    resident_half<T, L, NT, MQ, 0, 2>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
                else
                    resident_half<T, L, NT, MQ, 1, 2>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, tid);
            }
            __syncthreads();
        }
        if (need_e) {
            const double tot = block_sum<NT>(acc, red);
            if (tid == 0) s_H = -tot;
            __syncthreads();
            H = s_H;
        }
    }
    if (bad || !isfinite(H)) atomicOr(e.guard, 1);

    // write the replica back (regular) or to the candidate buffer (annealing)
    T* dstp = anneal ? reinterpret_cast<T*>(scr + sl.cand) + static_cast<size_t>(slot) * 3 * N : gs;
    {
        const uint4* src = reinterpret_cast<const uint4*>(sh);
        uint4* dst = reinterpret_cast<uint4*>(dstp);
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
        for (int v = tid; v < NV; v += NT) dst[v] = src[v];
    }
    if (tid == 0) {
        if (anneal) {
            e.work[(static_cast<size_t>(ch) * (R - 1) + ipair) * 2 + leg] = W;
            reinterpret_cast<double*>(scr + sl.cand_energy)[slot] = H;
            e.sweep_ctr[slot] = t0 + static_cast<uint32_t>(K);
        } else {
            e.energy[slot] = H;
            e.sweep_ctr[slot] = t0 + static_cast<uint32_t>(n_sweeps);
        }
    }
}

}  // namespace hsg
