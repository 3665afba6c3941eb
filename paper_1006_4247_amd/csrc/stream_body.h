// Device code of the streaming half-sweeps, shared by their kernels
// (sweep_stream.hip) and the persistent batch kernel (sweep_batch.hip).
#pragma once

#include "hsg_device.h"

namespace hsg {

struct StreamArgs {
    int hb[2], par[2], hs[2];  // per leg (regular sweeps use index 0)
    int rn[2];                 // renormalise the updated spins (sweeps without heat-bath)
    int step;                  // sweep index within the call / annealing step k
    int want;                  // 1: last half-sweep of a sweep, reduce energy
    int anneal, parity;        // annealing legs of pairs with i mod 2 == parity
    int n_tiles;
    double* partial;           // per-tile energies [slots][max_tiles] (see scratch_layout)
};

struct LegInfo {
    int slot, leg, ipair, K, ch;
};

__device__ __forceinline__ LegInfo leg_of_block(const hsg_ensemble& e, int b, int parity) {
    const int R = e.n_temps;
    const int npp = (R - parity) / 2;
    LegInfo li;
    li.leg = b & 1;
    const int rest = b >> 1;
    li.ch = rest / npp;
    li.ipair = parity + 2 * (rest % npp);
    li.slot = li.ch * R + label(e.slot_of_temp[li.ch * R + li.ipair + li.leg], R, e.guard);
    int K = e.anneal_K[li.ipair];
    if (K < 0) K = 0;
    if (K > e.anneal_K_max) K = e.anneal_K_max;
    li.K = K;
    return li;
}

__device__ __forceinline__ double proto(const hsg_ensemble& e, int ipair, int K, int k) {
    const double a = e.betas[ipair], b = e.betas[ipair + 1];
    if (k <= 0) return a;
    if (k >= K + 1) return b;
    if (e.anneal_lambda) return e.anneal_lambda[static_cast<size_t>(ipair) * e.anneal_K_max + (k - 1)];
    return a + static_cast<double>(k) * (b - a) / static_cast<double>(K + 1);
}

// One work item of a half-sweep: tile `tile` of the replica group `group` (`red`:
// workgroup-shared scratch of >= NT/64 doubles).  Used by k_stream_half and by the
// persistent batch kernel (sweep_batch.hip).
template <typename T, int LT, int NT, int RB>
__device__ __forceinline__ void stream_tile(const hsg_ensemble& e, const StreamArgs& a, int tile, int group,
                                            double* red) {
    const int L = LT > 0 ? LT : e.L;
    const int N = L * L * L, NH = N / 2, NQ = N / 4;
    const int C = e.n_chains, R = e.n_temps;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const int q = tile * NT + static_cast<int>(threadIdx.x);
    const bool active = q < NQ;

    int slot0, leg = 0, K = 0, ipair = 0;
    if (!a.anneal) {
        slot0 = group * RB;
    } else {
        const LegInfo li = leg_of_block(e, group, a.parity);
        if (a.step >= li.K) return;  // uniform over the block
        slot0 = li.slot;
        leg = li.leg;
        K = li.K;
        ipair = li.ipair;
    }
    const int hb = a.hb[leg], P = a.par[leg], hs = a.hs[leg], rn = a.rn[leg];
    const int smp = slot0 / (C * R);
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* base = a.anneal ? reinterpret_cast<T*>(scr + sl.cand) : static_cast<T*>(e.spins);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const uint32_t c3 = heatbath_c3(hs);

    int nb[2][6];
    T jr[2][6];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int h = (active ? q : 0) + half * NQ;
        const Nbr n = neighbours<LT>(h, P, L);
#pragma unroll
        for (int d = 0; d < 6; ++d) nb[half][d] = n.n[d];
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            jr[half][2 * mu] = J[(mu * 2 + P) * NH + h];
            jr[half][2 * mu + 1] = J[(mu * 2 + (1 - P)) * NH + n.n[2 * mu + 1]];
        }
    }

    for (int rb = 0; rb < RB; ++rb) {
        const int slot = slot0 + rb;
        if (!a.anneal && slot >= (slot0 / (C * R) + 1) * (C * R)) break;  // uniform
        double beta_d;
        if (a.anneal) {
            const int kk = a.step;  // sweep at protocol point k+1 (up) / K-k (down)
            beta_d = leg == 0 ? proto(e, ipair, K, kk + 1) : proto(e, ipair, K, K - kk);
        } else {
            beta_d = e.betas[label(e.temp_of_slot[slot], R, e.guard)];
        }
        const T beta = static_cast<T>(beta_d);
        const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
        const uint32_t tsw = e.sweep_ctr[slot] + static_cast<uint32_t>(a.step);
        T* sp = base + static_cast<size_t>(slot) * 3 * N;
        const T* __restrict__ o0 = sp + (0 * 2 + (1 - P)) * NH;
        const T* __restrict__ o1 = sp + (1 * 2 + (1 - P)) * NH;
        const T* __restrict__ o2 = sp + (2 * 2 + (1 - P)) * NH;
        T* w0 = sp + (0 * 2 + P) * NH;
        T* w1 = sp + (1 * 2 + P) * NH;
        T* w2 = sp + (2 * 2 + P) * NH;
        double acc = 0.0;
        bool bad = false;
        if (active) {
            Words wq{0, 0, 0, 0};
            if (sizeof(T) == 4 && hb) wq = philox(static_cast<uint32_t>(q), tsw, g, c3, k0, k1);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int h = q + half * NQ;
                T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const int idx = nb[half][d];
                    Sx = fma(jr[half][d], o0[idx], Sx);
                    Sy = fma(jr[half][d], o1[idx], Sy);
                    Sz = fma(jr[half][d], o2[idx], Sz);
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
                if (a.want) {
                    const double dx = ox, dy = oy, dz = oz;
                    acc += fma(dz, static_cast<double>(Sz),
                               fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
                    const double n2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    if (!(fabs(n2 - 1.0) <= NormTol<T>::value)) bad = true;
                }
            }
        }
        if (a.want) {
            if (bad) atomicOr(e.guard, 1);
            const double tot = block_sum<NT>(acc, red);
            if (threadIdx.x == 0)
                a.partial[static_cast<size_t>(slot) * sl.max_tiles + tile] = -tot;
        }
    }
}

}  // namespace hsg
