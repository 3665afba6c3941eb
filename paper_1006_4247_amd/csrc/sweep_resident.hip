// LDS-resident sweep kernels.
//
// One workgroup owns one replica: its whole lattice [3][2][N/2] sits in LDS for
// every half-sweep of the launch (n sweeps of a regular step, or the K sweeps
// of an annealing leg), so HBM sees one read and one write of the replica per
// launch.  Each thread owns fixed site pairs (h, h + N/4) of both sublattices
// and keeps their six couplings and six neighbour offsets in registers.  Sites
// of one sublattice never interact (paper Sec. III.A), so a half-sweep is one
// barrier-separated LDS pass; the energy H = -sum_{x in p} s_x.S_x is fused
// into the last half-sweep of each sweep (every bond has one end in p).
#include "hsg_device.h"
#include "hsg_launch.h"

namespace hsg {

template <typename T, int MQ>
struct Owned {
    int nb[2][MQ][2][6];  // [parity][pair][half][direction] neighbour index
    T j[2][MQ][2][6];     // matching couplings
};

// One half-sweep over the sites of parity P (compile-time), HB or OR.
template <typename T, int L, int NT, int MQ, int P>
__device__ __forceinline__ void resident_half(T* __restrict__ sh, const Owned<T, MQ>& own,
                                              bool hb, int hs, T beta, uint32_t tsw, uint32_t g,
                                              uint32_t k0, uint32_t k1, bool want,
                                              double& acc, bool& bad) {
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
    const T* __restrict__ o0 = sh + (0 * 2 + (1 - P)) * NH;
    const T* __restrict__ o1 = sh + (1 * 2 + (1 - P)) * NH;
    const T* __restrict__ o2 = sh + (2 * 2 + (1 - P)) * NH;
    T* __restrict__ w0 = sh + (0 * 2 + P) * NH;
    T* __restrict__ w1 = sh + (1 * 2 + P) * NH;
    T* __restrict__ w2 = sh + (2 * 2 + P) * NH;
    const uint32_t c3 = heatbath_c3(hs);
#pragma unroll
    for (int m = 0; m < MQ; ++m) {
        const int q = static_cast<int>(threadIdx.x) + NT * m;
        if ((NQ % NT) != 0 && q >= NQ) break;
        Words wq{0, 0, 0, 0};
        if (sizeof(T) == 4 && hb) wq = philox(static_cast<uint32_t>(q), tsw, g, c3, k0, k1);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int h = q + half * NQ;
            T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int idx = own.nb[P][m][half][d];
                const T jj = own.j[P][m][half][d];
                Sx = fma(jj, o0[idx], Sx);
                Sy = fma(jj, o1[idx], Sy);
                Sz = fma(jj, o2[idx], Sz);
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
            }
            w0[h] = ox;
            w1[h] = oy;
            w2[h] = oz;
            if (want) {
                const double dx = ox, dy = oy, dz = oz;
                acc += dx * static_cast<double>(Sx) + dy * static_cast<double>(Sy) +
                       dz * static_cast<double>(Sz);
                const double n2 = dx * dx + dy * dy + dz * dz;
                if (!(fabs(n2 - 1.0) <= NormTol<T>::value)) bad = true;
            }
        }
    }
}

// mode 0: regular sweeps of slot blockIdx.x at its own temperature.
// mode 1: annealing legs of the pairs with i mod 2 == parity; block ->
//         (chain, pair, leg); leg 0 = up (forward order), 1 = down (adjoint).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT)
    k_resident(hsg_ensemble e, int n_sweeps, int n_hb, int n_or, int anneal, int parity) {
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
    constexpr int MQ = (NQ + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sh = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[(NT + 63) / 64];
    __shared__ double s_H;

    const int C = e.n_chains, R = e.n_temps;
    int slot, leg = 0, ipair = 0, K = n_sweeps, ch = 0;
    double lam_a = 0.0, lam_b = 0.0;
    const double* lam_tab = nullptr;
    if (!anneal) {
        slot = blockIdx.x;
    } else {
        const int npp = (R - parity) / 2;
        leg = blockIdx.x & 1;
        const int rest = blockIdx.x >> 1;
        ch = rest / npp;
        ipair = parity + 2 * (rest % npp);
        slot = ch * R + label(e.slot_of_temp[ch * R + ipair + leg], R, e.guard);
        K = e.anneal_K[ipair];
        if (K < 0 || K > e.anneal_K_max) {
            if (threadIdx.x == 0) atomicOr(e.guard, 2);
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
        if (threadIdx.x == 0) {
            const double W = leg == 0 ? (lam_b - lam_a) * H : (lam_a - lam_b) * H;
            e.work[(static_cast<size_t>(ch) * (R - 1) + ipair) * 2 + leg] = W;
            reinterpret_cast<double*>(scr + sl.cand_energy)[slot] = H;
        }
        return;
    }

    // stage the replica into LDS (16-byte vectors)
    {
        const uint4* src = reinterpret_cast<const uint4*>(gs);
        uint4* dst = reinterpret_cast<uint4*>(sh);
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
        for (int v = threadIdx.x; v < NV; v += NT) dst[v] = src[v];
    }
    Owned<T, MQ> own;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int m = 0; m < MQ; ++m)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int q = static_cast<int>(threadIdx.x) + NT * m;
                const int h = (q < NQ ? q : 0) + half * NQ;
                const Nbr nb = neighbours<L>(h, p, L);
#pragma unroll
                for (int d = 0; d < 6; ++d) own.nb[p][m][half][d] = nb.n[d];
#pragma unroll
                for (int mu = 0; mu < 3; ++mu) {
                    own.j[p][m][half][2 * mu] = J[(mu * 2 + p) * NH + h];
                    own.j[p][m][half][2 * mu + 1] = J[(mu * 2 + (1 - p)) * NH + nb.n[2 * mu + 1]];
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
            const int p = pos & 1;
            const bool want = need_e && (step == nhalf - 1);
            if (p == 0)
                resident_half<T, L, NT, MQ, 0>(sh, own, hb, pos, beta, tsw, g, k0, k1, want, acc, bad);
            else
                resident_half<T, L, NT, MQ, 1>(sh, own, hb, pos, beta, tsw, g, k0, k1, want, acc, bad);
            __syncthreads();
        }
        if (need_e) {
            const double tot = block_sum<NT>(acc, red);
            if (threadIdx.x == 0) s_H = -tot;
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
        for (int v = threadIdx.x; v < NV; v += NT) dst[v] = src[v];
    }
    if (threadIdx.x == 0) {
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

// ---------------------------------------------------------------- dispatch
static int default_threads(int L) {
    const int NQ = L * L * L / 4;
    int nt = ((NQ + 63) / 64) * 64;
    if (nt > 1024) nt = 1024;
    return nt;
}

size_t max_block_lds() {
    static size_t cached = 0;
    if (cached == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cached = prop.sharedMemPerBlock;
        if (cached == 0) cached = 65536;
    }
    return cached;
}

template <typename T, int L, int NT>
static hipError_t go(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                     int parity, hipStream_t st) {
    constexpr int N = L * L * L;
    const size_t lds = 3 * N * sizeof(T);
    const int R = e.n_temps;
    const int chains = e.n_samples * e.n_chains;
    int blocks;
    if (!anneal)
        blocks = chains * R;
    else
        blocks = chains * ((R - parity) / 2) * 2;
    if (blocks <= 0) return hipSuccess;
    auto kern = k_resident<T, L, NT>;
    if (lds > 65536) {
        hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (a != hipSuccess) return a;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or, anneal,
                       parity);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t go_nt(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                        int parity, int nt, hipStream_t st) {
    constexpr int NQ = L * L * L / 4;
    constexpr int DEF = ((NQ + 63) / 64) * 64 > 1024 ? 1024 : ((NQ + 63) / 64) * 64;
    if (nt == 0 || nt == DEF) return go<T, L, DEF>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
    if constexpr (DEF >= 512) {
        if (nt == 512) return go<T, L, 512>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
        if (nt == 256) return go<T, L, 256>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t dispatch(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                           int parity, int nt, hipStream_t st) {
    switch (e.L) {
    case 2: return go_nt<T, 2>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 4: return go_nt<T, 4>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 6: return go_nt<T, 6>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 8: return go_nt<T, 8>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 10: return go_nt<T, 10>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 12: return go_nt<T, 12>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 14: return go_nt<T, 14>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    case 16: return go_nt<T, 16>(e, n_sweeps, n_hb, n_or, anneal, parity, nt, st);
    default: return hipErrorInvalidValue;
    }
}

bool resident_supported(const hsg_ensemble& e) {
    if (e.L < 2 || e.L > 16 || (e.L & 1)) return false;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const size_t lds = 3 * N * (e.precision == HSG_FP64 ? 8 : 4);
    return lds <= max_block_lds();
}

hipError_t launch_resident(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                           int parity, int block_threads, hipStream_t st) {
    (void)default_threads;
    if (e.precision == HSG_FP64)
        return dispatch<double>(e, n_sweeps, n_hb, n_or, anneal, parity, block_threads, st);
    return dispatch<float>(e, n_sweeps, n_hb, n_or, anneal, parity, block_threads, st);
}

}  // namespace hsg
