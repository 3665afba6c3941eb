// LDS-resident sweep kernels.
//
// One workgroup owns one replica: its whole lattice [3][2][N/2] sits in LDS for
// every half-sweep of the launch (n sweeps of a regular step, or the K sweeps
// of an annealing leg), so HBM sees one read and one write of the replica per
// launch.  Each thread owns fixed site pairs (h, h + N/4) of both sublattices
// and keeps their six couplings in registers (neighbour offsets are recomputed).  Sites
// of one sublattice never interact (paper Sec. III.A), so a half-sweep is one
// barrier-separated LDS pass; the energy H = -sum_{x in p} s_x.S_x is fused
// into the last half-sweep of each sweep (every bond has one end in p).
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "hsg_device.h"
#include "hsg_launch.h"
#include "resident_body.h"

namespace hsg {

// Regular sweeps: one workgroup per replica.  Annealing legs run the same steps in
// k_resident_leg; a kernel of their own keeps the legs' protocol state out of the
// regular sweep's registers (102 against 115 VGPRs at binary32 L = 16).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_resident(hsg_ensemble e, int n_sweeps, int n_hb, int n_or) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[(NT + 63) / 64];
    __shared__ double s_H;
    resident_item<T, L, NT>(e, xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x)), n_sweeps,
                            n_hb, n_or, 0, 0, smem_raw, red, s_H);
}

// Annealing legs of the pairs i = parity (mod 2): one workgroup per (chain, pair, leg).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_resident_leg(hsg_ensemble e, int n_hb, int n_or, int parity) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[(NT + 63) / 64];
    __shared__ double s_H;
    resident_item<T, L, NT>(e, xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x)), 0,
                            n_hb, n_or, 1, parity, smem_raw, red, s_H);
}

// Regular sweeps and the measurement of one (sample, temperature) in one launch, for
// ensembles of two chains: workgroup of 2 NT threads, threads [0, NT) running chain
// 0's replica at that temperature and [NT, 2 NT) chain 1's, each half taking exactly
// the steps of k_resident<T, L, NT> on its replica (same site order, random numbers
// and energy reduction, hence the same spins and energy bit for bit).  With both
// final configurations in LDS the workgroup then measures that temperature: the
// energy per site of both chains, the overlap tensor Q^{mu nu} = sum_x s1^mu(x)
// s2^nu(x) and chi = (1/N) sum Q^2 (paper Sec. IV), so the measurement reads no
// spins from HBM.
template <typename T, int L, int NT>
__global__ void __launch_bounds__(2 * NT)
    k_resident_pair(hsg_ensemble e, int n_sweeps, int n_hb, int n_or) {
    static_assert(NT % 64 == 0, "each half of the workgroup is a whole number of waves");
    constexpr int N = L * L * L, NQ = N / 4;
    constexpr int MQ = (NQ + NT - 1) / NT;
    constexpr int NW = NT / 64;  // waves per replica
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[9 * 2 * NW];
    __shared__ double s_H[2];

    const int rep = static_cast<int>(threadIdx.x) >= NT ? 1 : 0;
    const int t = static_cast<int>(threadIdx.x) - rep * NT;
    T* sh = reinterpret_cast<T*>(smem_raw) + rep * 3 * N;
    const int R = e.n_temps;
    const int item = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int smp = item / R, b = item - smp * R;
    const int chain = smp * 2 + rep;
    const int slot = chain * R + label(e.slot_of_temp[chain * R + b], R, e.guard);
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* gs = static_cast<T*>(e.spins) + static_cast<size_t>(slot) * 3 * N;
    const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
    const uint32_t t0 = e.sweep_ctr[slot];
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);

    // couplings and replica into LDS, as in k_resident (regular sweeps)
    Owned<T, MQ> own;
    const FirstNbr fn = first_neighbours<L, NT>(t);
    {
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
        constexpr int NVP = NV / 6;
        constexpr int PV = (NV + NT - 1) / NT;
        constexpr bool PREFETCH = PV <= 6;
        const bool hb_first = n_hb > 0;
        const uint4* js = reinterpret_cast<const uint4*>(J);
        const uint4* src = reinterpret_cast<const uint4*>(gs);
        uint4* dst = reinterpret_cast<uint4*>(sh);
        const int n_load = hb_first ? NV / 2 : NV;
        if constexpr (PREFETCH) {
            uint4 jv[PV], sv[PV];
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = t + k * NT;
                jv[k] = (v < NV) ? js[v] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = t + k * NT;
                sv[k] = (v < n_load) ? src[loaded_vec<NVP>(v, hb_first)] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = t + k * NT;
                if (v < NV) dst[v] = jv[k];
            }
            lds_barrier();
            load_owned<T, L, NT, MQ>(own, sh, fn, t);
            lds_barrier();
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int v = t + k * NT;
                if (v < n_load) dst[loaded_vec<NVP>(v, hb_first)] = sv[k];
            }
        } else {
            for (int v = t; v < NV; v += NT) dst[v] = js[v];
            __syncthreads();
            load_owned<T, L, NT, MQ>(own, sh, fn, t);
            __syncthreads();
            for (int v = t; v < n_load; v += NT) {
                const int o = loaded_vec<NVP>(v, hb_first);
                dst[o] = src[o];
            }
        }
    }
    __syncthreads();

    const int nhalf = 2 * (n_hb + n_or);
    const T beta = static_cast<T>(e.betas[label(e.temp_of_slot[slot], R, e.guard)]);
    double H = 0.0;
    bool bad = false;
    for (int k = 0; k < n_sweeps; ++k) {
        const bool need_e = k == n_sweeps - 1;
        const uint32_t tsw = t0 + static_cast<uint32_t>(k);
        double acc = 0.0;
        for (int step = 0; step < nhalf; ++step) {
            const bool hb = step < 2 * n_hb;
            const bool rn = renorm_on(e) && n_hb == 0 && step >= nhalf - 2;
            const bool want = need_e && (step == nhalf - 1);
            if ((step & 1) == 0)
                resident_half<T, L, NT, MQ, 0>(sh, own, fn, hb, rn, step, beta, tsw, g, k0, k1, want, acc, bad, t);
            else
                resident_half<T, L, NT, MQ, 1>(sh, own, fn, hb, rn, step, beta, tsw, g, k0, k1, want, acc, bad, t);
            __syncthreads();
        }
        if (need_e) {  // each half sums its own waves, in wave order
            const double w = wave_sum(acc);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
            __syncthreads();
            if (t == 0) {
                double s = 0.0;
#pragma unroll
                for (int v = 0; v < NW; ++v) s += red[rep * NW + v];
                s_H[rep] = -s;
            }
            __syncthreads();
            H = s_H[rep];
        }
    }
    if (bad || !isfinite(H)) atomicOr(e.guard, 1);
    {
        const uint4* src = reinterpret_cast<const uint4*>(sh);
        uint4* dst = reinterpret_cast<uint4*>(gs);
        constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;
        for (int v = t; v < NV; v += NT) dst[v] = src[v];
    }
    if (t == 0) {
        e.energy[slot] = H;
        e.sweep_ctr[slot] = t0 + static_cast<uint32_t>(n_sweeps);
        e.e_temp[static_cast<size_t>(chain) * R + b] = H / static_cast<double>(N);
    }

    // overlap of the two replicas, site by site in the common LDS layout [3][2][N/2]
    const T* a = reinterpret_cast<const T*>(smem_raw);
    const T* c = a + 3 * N;
    double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = static_cast<int>(threadIdx.x); x < N; x += 2 * NT) {
        const double x0 = a[x], x1 = a[N + x], x2 = a[2 * N + x];
        const double y0 = c[x], y1 = c[N + x], y2 = c[2 * N + x];
        q[0] = fma(x0, y0, q[0]); q[1] = fma(x0, y1, q[1]); q[2] = fma(x0, y2, q[2]);
        q[3] = fma(x1, y0, q[3]); q[4] = fma(x1, y1, q[4]); q[5] = fma(x1, y2, q[5]);
        q[6] = fma(x2, y0, q[6]); q[7] = fma(x2, y1, q[7]); q[8] = fma(x2, y2, q[8]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double w = wave_sum(q[k]);
        if ((threadIdx.x & 63) == 0) red[k * 2 * NW + (threadIdx.x >> 6)] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double chi = 0.0;
        for (int k = 0; k < 9; ++k) {
            double s = 0.0;
            for (int v = 0; v < 2 * NW; ++v) s += red[k * 2 * NW + v];
            e.Q[(static_cast<size_t>(smp) * R + b) * 9 + k] = s;
            chi += s * s;
        }
        e.chi[static_cast<size_t>(smp) * R + b] = chi / static_cast<double>(N);
    }
}

// Regular sweeps and the measurement of one (sample, temperature), ensembles of two
// chains, binary32 L = 16 with 512 threads per replica: the workgroup sweeps the chain-0
// replica at that temperature and then the chain-1 replica, each exactly as k_resident
// does (same site order, random numbers and energy reduction, hence the same spins and
// energies bit for bit), and measures the pair as the measurement pass does: e = H/N
// of both, Q^{mu nu} = sum_x s1^mu(x) s2^nu(x) and chi = (1/N) sum Q^2 (paper Sec. IV),
// from the chain-1 replica still in LDS and the chain-0 replica read back — each thread
// reads the 16-byte vectors it wrote itself, one position of every plane, so its own
// writes are all it needs to see.  This saves the measurement pass's second read of
// every replica; Q is summed in another order (within rounding of the pass's).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_resident_mseq(hsg_ensemble e, int n_sweeps, int n_hb, int n_or) {
    constexpr int N = L * L * L;
    constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per replica
    constexpr int NVP = NV / 6;                                    // per plane [component][parity]
    constexpr int W = 16 / static_cast<int>(sizeof(T));            // sites per vector
    static_assert(NVP == NT, "each thread holds the same position of every plane");
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[9 * NW];
    __shared__ double s_H;
    const int R = e.n_temps;
    const int t = static_cast<int>(threadIdx.x);
    const int item = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int smp = item / R, b = item - smp * R;
    int slots[2];
    double H[2];
    Owned<T, (N / 4 + NT - 1) / NT> own;  // both replicas belong to one sample: couplings loaded once
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
        const int chain = smp * 2 + rep;
        slots[rep] = chain * R + label(e.slot_of_temp[chain * R + b], R, e.guard);
        // overrelaxation half-sweeps as one block each, heat-bath ones from the general
        // form: measured 0.129 ms per launch at 64 x 2 x 24, against 0.131 ms with both
        // kinds fixed (and an opaque thread index per replica to hold 115 VGPRs)
        if (rep == 0)
            resident_item<T, L, NT, 1, 2>(e, slots[rep], n_sweeps, n_hb, n_or, 0, 0, smem_raw, red, s_H, &own);
        else
            resident_item<T, L, NT, 2, 2>(e, slots[rep], n_sweeps, n_hb, n_or, 0, 0, smem_raw, red, s_H, &own);
        H[rep] = s_H;  // written before the energy's barrier
        // every thread has read it and the write-back has read the LDS; its stores stay
        // in flight (a thread's later reads of its own writes see them)
        lds_barrier();
    }
    if (t == 0) {
        e.e_temp[(static_cast<size_t>(smp) * 2 + 0) * R + b] = H[0] / static_cast<double>(N);
        e.e_temp[(static_cast<size_t>(smp) * 2 + 1) * R + b] = H[1] / static_cast<double>(N);
    }
    struct alignas(16) Vec { T v[W]; };
    const Vec* a = reinterpret_cast<const Vec*>(static_cast<const T*>(e.spins) + static_cast<size_t>(slots[0]) * 3 * N);
    const Vec* c = reinterpret_cast<const Vec*>(smem_raw);
    Vec av[6], cv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {  // plane k = 2 mu + parity, position t
        av[k] = a[k * NVP + t];
        cv[k] = c[k * NVP + t];
    }
    double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double x0 = av[0 + p].v[w], x1 = av[2 + p].v[w], x2 = av[4 + p].v[w];
            const double y0 = cv[0 + p].v[w], y1 = cv[2 + p].v[w], y2 = cv[4 + p].v[w];
            q[0] = fma(x0, y0, q[0]); q[1] = fma(x0, y1, q[1]); q[2] = fma(x0, y2, q[2]);
            q[3] = fma(x1, y0, q[3]); q[4] = fma(x1, y1, q[4]); q[5] = fma(x1, y2, q[5]);
            q[6] = fma(x2, y0, q[6]); q[7] = fma(x2, y1, q[7]); q[8] = fma(x2, y2, q[8]);
        }
    // the nine sums: every thread's partials into LDS (over the replica, now read),
    // then wave w adds up component k = w (and k = 8 for wave 0): each lane the
    // partials of threads lane, lane + 64, ..., then a butterfly over the lanes
    double* part = reinterpret_cast<double*>(smem_raw);  // [9][NT]
    lds_barrier();  // every thread has read its replica vectors
#pragma unroll
    for (int k = 0; k < 9; ++k) part[k * NT + t] = q[k];
    lds_barrier();
    const int wv = t >> 6, lane = t & 63;
    for (int k = wv; k < 9; k += NW) {
        double u = 0.0;
#pragma unroll
        for (int j = lane; j < NT; j += 64) u += part[k * NT + j];
        u = wave_sum(u);
        if (lane == 0) red[k] = u;
    }
    lds_barrier();
    if (t == 0) {
        double chi = 0.0;
        for (int k = 0; k < 9; ++k) {
            e.Q[(static_cast<size_t>(smp) * R + b) * 9 + k] = red[k];
            chi += red[k] * red[k];
        }
        e.chi[static_cast<size_t>(smp) * R + b] = chi / static_cast<double>(N);
    }
}

// Persistent variant for regular sweeps: each workgroup takes a contiguous range
// of slots (consecutive replicas mostly share a sample, whose couplings then stay
// in registers) and double-buffers the replicas in LDS: the next replica's loads
// are issued during the current replica's overrelaxation half-sweeps and the
// finished replica's stores drain behind the next one, so the load/store phases
// overlap the arithmetic.  Its barriers are LDS-only (lds_barrier) so that those
// global accesses stay in flight across them.
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT)
    k_resident_persist(hsg_ensemble e, int n_sweeps, int n_hb, int n_or, int n_tasks) {
    constexpr int N = L * L * L, NQ = N / 4;
    constexpr int MQ = (NQ + NT - 1) / NT;
    constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per replica
    constexpr int PF = (NV + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint4* buf0 = reinterpret_cast<uint4*>(smem_raw);
    uint4* buf1 = buf0 + NV;
    __shared__ double red[(NT + 63) / 64];
    __shared__ double s_H;

    const int C = e.n_chains, R = e.n_temps;
    const long long bid = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int t_begin = static_cast<int>(bid * n_tasks / gridDim.x);
    const int t_end = static_cast<int>((bid + 1) * n_tasks / gridDim.x);
    if (t_begin >= t_end) return;
    const uint4* gsrc = static_cast<const uint4*>(e.spins);
    uint4* gdst = static_cast<uint4*>(e.spins);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int nhalf = 2 * (n_hb + n_or);

    for (int v = threadIdx.x; v < NV; v += NT) buf0[v] = gsrc[static_cast<size_t>(t_begin) * NV + v];
    int cur_sample = -1;
    Owned<T, MQ> own;
    const FirstNbr fn = first_neighbours<L, NT>(static_cast<int>(threadIdx.x));
    uint4 pf[PF];
    int sel = 0;
    for (int slot = t_begin; slot < t_end; ++slot) {
        T* sh = reinterpret_cast<T*>(sel ? buf1 : buf0);
        uint4* nxt = sel ? buf0 : buf1;
        const int smp = slot / (C * R);
        if (smp != cur_sample) {
            const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
            load_owned<T, L, NT, MQ>(own, J, fn, static_cast<int>(threadIdx.x));
            cur_sample = smp;
        }
        const bool has_next = slot + 1 < t_end;
        lds_barrier();  // this replica is in LDS; the other buffer's readers are done

        const T beta = static_cast<T>(e.betas[label(e.temp_of_slot[slot], R, e.guard)]);
        const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
        const uint32_t t0 = e.sweep_ctr[slot];
        double H = 0.0;
        bool bad = false;
        // Sweeps before the last one, then the last sweep split so that the next
        // replica's loads are issued after its heat-bath half-sweeps (outside the
        // heat-bath's register peak) and land during the overrelaxation ones.
        double acc = 0.0;
        const int n_pre = (n_or > 0) ? 2 * n_hb : nhalf - 1;  // half-sweeps before the loads
        for (int k = 0; k < n_sweeps; ++k) {
            const bool last = (k == n_sweeps - 1);
            const uint32_t tsw = t0 + static_cast<uint32_t>(k);
            const int stop = last ? n_pre : nhalf;
            for (int pos = 0; pos < stop; ++pos) {
                const bool hb = pos < 2 * n_hb;
                const bool rn = renorm_on(e) && n_hb == 0 && pos >= nhalf - 2;
                if ((pos & 1) == 0)
                    resident_half<T, L, NT, MQ, 0>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, false, acc, bad, static_cast<int>(threadIdx.x));
                else
                    resident_half<T, L, NT, MQ, 1>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, false, acc, bad, static_cast<int>(threadIdx.x));
                lds_barrier();
            }
        }
        if (has_next) {
#pragma unroll
            for (int kk = 0; kk < PF; ++kk) {
                const int v = static_cast<int>(threadIdx.x) + kk * NT;
                pf[kk] = (v < NV) ? gsrc[static_cast<size_t>(slot + 1) * NV + v] : make_uint4(0, 0, 0, 0);
            }
        }
        {
            const uint32_t tsw = t0 + static_cast<uint32_t>(n_sweeps - 1);
            for (int pos = n_pre; pos < nhalf; ++pos) {
                const bool hb = pos < 2 * n_hb;
                const bool rn = renorm_on(e) && n_hb == 0 && pos >= nhalf - 2;
                const bool want = pos == nhalf - 1;
                if ((pos & 1) == 0)
                    resident_half<T, L, NT, MQ, 0>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, static_cast<int>(threadIdx.x));
                else
                    resident_half<T, L, NT, MQ, 1>(sh, own, fn, hb, rn, pos, beta, tsw, g, k0, k1, want, acc, bad, static_cast<int>(threadIdx.x));
                lds_barrier();
            }
        }
        {
            const double tot = block_sum<NT, true>(acc, red);
            if (threadIdx.x == 0) s_H = -tot;
            lds_barrier();
            H = s_H;
        }
        if (bad || !isfinite(H)) atomicOr(e.guard, 1);
        const uint4* shv = reinterpret_cast<const uint4*>(sh);
        for (int v = threadIdx.x; v < NV; v += NT) gdst[static_cast<size_t>(slot) * NV + v] = shv[v];
        if (has_next) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int v = static_cast<int>(threadIdx.x) + k * NT;
                if (v < NV) nxt[v] = pf[k];
            }
        }
        if (threadIdx.x == 0) {
            e.energy[slot] = H;
            e.sweep_ctr[slot] = t0 + static_cast<uint32_t>(n_sweeps);
        }
        sel ^= 1;
    }
}

// Persistent variant with a replica buffer and a staging area, for regular sweeps
// that open with a heat-bath half-sweep of parity 0 (which reads no parity-0 spin,
// so only the three parity-1 planes of a replica are loaded): each workgroup takes a
// contiguous range of slots, which share a sample (and its couplings, kept in
// registers) whenever the range lies within one.  While a replica is swept, the next
// one's parity-1 planes travel from HBM straight into the staging area (loads that
// write the LDS without passing through registers); after the write-back they are
// copied into the replica buffer.  48 KB + 24 KB of LDS let two 512-thread
// workgroups share a CU, as with k_resident.  Every half-sweep is the one k_resident
// takes, so spins are bit for bit the same; the energy is the same reduction.
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT)
    k_resident_chain(hsg_ensemble e, int n_sweeps, int n_hb, int n_or, int n_tasks) {
    constexpr int N = L * L * L, NQ = N / 4;
    constexpr int MQ = (NQ + NT - 1) / NT;
    constexpr int NV = 3 * N * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per replica
    constexpr int NVP = NV / 6;                                    // per plane
    constexpr int NL = NV / 2;                                     // loaded: the parity-1 planes
    static_assert(NL % NT == 0 && NT % 64 == 0, "whole waves of staged vectors");
    constexpr int PF = NL / NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ uint4 stage[NL];
    uint4* buf = reinterpret_cast<uint4*>(smem_raw);
    T* sh = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[(NT + 63) / 64];
    __shared__ double s_H;

    const int C = e.n_chains, R = e.n_temps;
    const long long bid = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int t_begin = static_cast<int>(bid * n_tasks / gridDim.x);
    const int t_end = static_cast<int>((bid + 1) * n_tasks / gridDim.x);
    if (t_begin >= t_end) return;
    const uint4* gsrc = static_cast<const uint4*>(e.spins);
    uint4* gdst = static_cast<uint4*>(e.spins);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int nhalf = 2 * (n_hb + n_or);
    const int t = static_cast<int>(threadIdx.x);
    const int wave_base = t & ~63;

    for (int v = t; v < NL; v += NT) {
        const int o = loaded_vec<NVP>(v, true);
        buf[o] = gsrc[static_cast<size_t>(t_begin) * NV + o];
    }
    int cur_sample = -1;
    Owned<T, MQ> own;
    const FirstNbr fn = first_neighbours<L, NT>(t);
    for (int slot = t_begin; slot < t_end; ++slot) {
        const int smp = slot / (C * R);
        if (smp != cur_sample) {
            const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
            load_owned<T, L, NT, MQ>(own, J, fn, t);
            cur_sample = smp;
        }
        const bool has_next = slot + 1 < t_end;
        // read before the staged loads go out: a wait for a later load waits for them too
        T beta = static_cast<T>(e.betas[label(e.temp_of_slot[slot], R, e.guard)]);
        asm volatile("" : "+v"(beta));  // converted here (no instruction emitted)
        const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
        const uint32_t t0 = e.sweep_ctr[slot];
        lds_barrier();  // this replica's parity-1 planes are in the buffer
        if (has_next) {
            // vector v = k NT + t of the staging area; a wave writes 64 consecutive ones
            const uint4* nsrc = gsrc + static_cast<size_t>(slot + 1) * NV;
#pragma unroll
            for (int k = 0; k < PF; ++k)
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void*>(nsrc + loaded_vec<NVP>(k * NT + t, true)),
                    (__attribute__((address_space(3))) void*)(stage + k * NT + wave_base), 16, 0, 0);
        }

        double acc = 0.0;
        bool bad = false;
        for (int k = 0; k < n_sweeps; ++k) {
            const bool last = (k == n_sweeps - 1);
            const uint32_t tsw = t0 + static_cast<uint32_t>(k);
            for (int pos = 0; pos < nhalf; ++pos) {
                const bool hb = pos < 2 * n_hb;
                const bool want = last && pos == nhalf - 1;
                if ((pos & 1) == 0)
                    resident_half<T, L, NT, MQ, 0>(sh, own, fn, hb, false, pos, beta, tsw, g, k0, k1, want, acc, bad, t);
                else
                    resident_half<T, L, NT, MQ, 1>(sh, own, fn, hb, false, pos, beta, tsw, g, k0, k1, want, acc, bad, t);
                lds_barrier();
            }
        }
        double H;
        {
            const double tot = block_sum<NT, true>(acc, red);
            if (t == 0) s_H = -tot;
            lds_barrier();
            H = s_H;
        }
        if (bad || !isfinite(H)) atomicOr(e.guard, 1);
        // this wave's staged loads have landed (issued a replica ago; waited for here,
        // before the write-back's stores join the same counter)
        __builtin_amdgcn_s_waitcnt(0x0F70);  // gfx9 encoding: vmcnt = 0, expcnt = 7, lgkmcnt = 15
        for (int v = t; v < NV; v += NT) gdst[static_cast<size_t>(slot) * NV + v] = buf[v];
        if (has_next) {
            lds_barrier();  // every wave's staging is complete and this replica has been read
#pragma unroll
            for (int k = 0; k < PF; ++k) buf[loaded_vec<NVP>(k * NT + t, true)] = stage[k * NT + t];
        }
        if (t == 0) {
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

// Per-device launch facts, filled on first use under a lock (the library may be
// called from several host threads and on several devices).
namespace {
struct DeviceFacts {
    size_t max_lds = 0;
    int cus = 0;
};
std::mutex g_facts_mu;
std::map<int, DeviceFacts> g_facts;
std::map<std::pair<const void*, int>, int> g_kernel_ok;  // (kernel, device) -> blocks per CU

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return dev;
}

DeviceFacts device_facts() {
    const int dev = current_device();
    std::lock_guard<std::mutex> lock(g_facts_mu);
    auto it = g_facts.find(dev);
    if (it != g_facts.end()) return it->second;
    DeviceFacts f;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        f.max_lds = prop.sharedMemPerBlock;
        f.cus = prop.multiProcessorCount;
    }
    if (f.max_lds == 0) f.max_lds = 65536;
    if (f.cus <= 0) f.cus = 256;
    g_facts[dev] = f;
    return f;
}
}  // namespace

size_t max_block_lds() { return device_facts().max_lds; }

static int num_cus() { return device_facts().cus; }

int device_cus() { return num_cus(); }

hipError_t allow_dynamic_lds(const void* kern, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    const std::pair<const void*, int> key(kern, current_device());
    std::lock_guard<std::mutex> lock(g_facts_mu);
    if (g_kernel_ok.count(key)) return hipSuccess;
    const hipError_t a = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(lds));
    if (a == hipSuccess) g_kernel_ok[key] = 0;
    return a;
}

// Workgroups of `kern` (NT threads, lds bytes) resident per CU, queried once per
// device (not per launch, so that launches can be captured into graphs without
// host-side queries in between).
hipError_t blocks_per_cu_query(const void* kern, int nt, size_t lds, int* out) {
    hipError_t a = allow_dynamic_lds(kern, lds);
    if (a != hipSuccess) return a;
    const std::pair<const void*, int> key(kern, current_device());
    std::lock_guard<std::mutex> lock(g_facts_mu);
    auto it = g_kernel_ok.find(key);
    if (it != g_kernel_ok.end() && it->second > 0) {
        *out = it->second;
        return hipSuccess;
    }
    int pc = 0;
    a = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, nt, lds);
    pc = (a != hipSuccess || pc < 1) ? 1 : pc;
    g_kernel_ok[key] = pc;
    *out = pc;
    return hipSuccess;
}

template <typename T, int L, int NT>
static hipError_t go_persist(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    constexpr int N = L * L * L;
    const size_t lds = 2 * 3 * N * sizeof(T);
    const int n_tasks = e.n_samples * e.n_chains * e.n_temps;
    auto kern = k_resident_persist<T, L, NT>;
    int per_cu = 1;
    hipError_t a = blocks_per_cu_query(reinterpret_cast<const void*>(kern), NT, lds, &per_cu);
    if (a != hipSuccess) return a;
    int grid = num_cus() * per_cu;
    if (grid > n_tasks) grid = n_tasks;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or, n_tasks);
    return hipGetLastError();
}

template <typename T, int L, int NT>
static hipError_t go(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                     int parity, hipStream_t st);

// One persistent workgroup per resident slot of the CUs, each sweeping a contiguous
// range of replicas (k_resident_chain); sweeps without a heat-bath half-sweep, which
// read both parities, go to k_resident (the same results).
template <typename T, int L, int NT>
static hipError_t go_chain(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    if (n_hb == 0) return go<T, L, NT>(e, n_sweeps, n_hb, n_or, 0, 0, st);
    constexpr int N = L * L * L;
    const size_t lds = 3 * N * sizeof(T);
    const int n_tasks = e.n_samples * e.n_chains * e.n_temps;
    if (n_tasks <= 0 || n_sweeps <= 0) return hipSuccess;
    auto kern = k_resident_chain<T, L, NT>;
    int per_cu = 1;
    hipError_t a = blocks_per_cu_query(reinterpret_cast<const void*>(kern), NT, lds, &per_cu);
    if (a != hipSuccess) return a;
    int grid = num_cus() * per_cu;
    if (grid > n_tasks) grid = n_tasks;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or, n_tasks);
    return hipGetLastError();
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
    if (!anneal) {
        auto kern = k_resident<T, L, NT>;
        hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
        if (a != hipSuccess) return a;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or);
    } else {
        auto kern = k_resident_leg<T, L, NT>;
        hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
        if (a != hipSuccess) return a;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, n_hb, n_or, parity);
    }
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t go_nt(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                        int parity, int nt, hipStream_t st) {
    constexpr int NQ = L * L * L / 4;
    constexpr int DEF = ((NQ + 63) / 64) * 64 > 1024 ? 1024 : ((NQ + 63) / 64) * 64;
    if (anneal == 2) {  // regular sweeps, persistent double-buffered workgroups
        if (nt == 0 || nt == DEF) return go_persist<T, L, DEF>(e, n_sweeps, n_hb, n_or, st);
        return hipErrorInvalidValue;
    }
    if (anneal == 3) {  // regular sweeps, persistent single-buffer workgroups
        if constexpr (std::is_same<T, float>::value && L == 16) {
            if (nt == 0 || nt == 512) return go_chain<T, L, 512>(e, n_sweeps, n_hb, n_or, st);
        }
        return hipErrorInvalidValue;
    }
    // default: one 512-thread workgroup per replica where a replica has >= 1024 site
    // pairs (two such workgroups share a CU and overlap each other's LDS staging),
    // else one thread per site pair
    if (nt == 0) {
        if constexpr (DEF >= 1024)
            return go<T, L, 512>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
        else
            return go<T, L, DEF>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
    }
    if (nt == DEF) return go<T, L, DEF>(e, n_sweeps, n_hb, n_or, anneal, parity, st);
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

template <typename T, int L>
static hipError_t go_pair(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    // per replica the default workgroup size of k_resident, at most 512 threads in
    // binary32 and 256 in binary64 (whose site updates need more than the 128
    // registers a thread of a 1024-thread workgroup gets)
    constexpr int NQ = L * L * L / 4;
    constexpr int DEF = ((NQ + 63) / 64) * 64;
    constexpr int CAP = sizeof(T) == 4 ? 512 : 256;
    constexpr int NT = DEF > CAP ? CAP : DEF;
    const size_t lds = 2 * 3 * static_cast<size_t>(L) * L * L * sizeof(T);
    const int blocks = e.n_samples * e.n_temps;
    if (blocks <= 0 || n_sweeps <= 0) return hipSuccess;
    auto kern = k_resident_pair<T, L, NT>;
    const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (a != hipSuccess) return a;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(2 * NT), lds, st, e, n_sweeps, n_hb, n_or);
    return hipGetLastError();
}

// Sizes where the one launch was measured faster than the sweep and measurement
// launches (binary32 L <= 10, binary64 L <= 12).  From binary32 L = 12 and binary64
// L = 14 up the single-replica sweep keeps more workgroups per CU, whose load and
// store phases overlap each other's arithmetic, and the two launches win (at
// binary32 L = 16: 0.149 ms against 0.187 ms per step).
constexpr int pair_max_L(bool fp64) { return fp64 ? 12 : 10; }

template <typename T>
static hipError_t dispatch_pair(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    switch (e.L) {
    case 2: return go_pair<T, 2>(e, n_sweeps, n_hb, n_or, st);
    case 4: return go_pair<T, 4>(e, n_sweeps, n_hb, n_or, st);
    case 6: return go_pair<T, 6>(e, n_sweeps, n_hb, n_or, st);
    case 8: return go_pair<T, 8>(e, n_sweeps, n_hb, n_or, st);
    case 10: return go_pair<T, 10>(e, n_sweeps, n_hb, n_or, st);
    case 12:
        if constexpr (sizeof(T) == 8) return go_pair<T, 12>(e, n_sweeps, n_hb, n_or, st);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

bool resident_supported(const hsg_ensemble& e) {
    if (e.L < 2 || e.L > 16 || (e.L & 1)) return false;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const size_t lds = 3 * N * (e.precision == HSG_FP64 ? 8 : 4);
    return lds <= max_block_lds();
}

bool persistent_supported(const hsg_ensemble& e) {
    if (!resident_supported(e)) return false;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    return 2 * 3 * N * (e.precision == HSG_FP64 ? 8 : 4) <= max_block_lds();
}

bool resident_pair_supported(const hsg_ensemble& e) {
    if (!resident_supported(e) || e.n_chains != 2 || !e.Q || !e.chi || !e.e_temp) return false;
    if (e.L > pair_max_L(e.precision == HSG_FP64)) return false;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    return 2 * 3 * N * (e.precision == HSG_FP64 ? 8 : 4) <= max_block_lds();
}

bool chain_supported(const hsg_ensemble& e) {
    return resident_supported(e) && e.precision == HSG_FP32 && e.L == 16;
}

bool resident_mseq_supported(const hsg_ensemble& e) {
    return resident_supported(e) && e.precision == HSG_FP32 && e.L == 16 && e.n_chains == 2 && e.Q && e.chi &&
           e.e_temp;
}

hipError_t launch_resident_mseq(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    constexpr int L = 16, NT = 512;
    const size_t lds = 3 * L * L * L * sizeof(float);
    const int blocks = e.n_samples * e.n_temps;
    if (blocks <= 0) return hipSuccess;
    auto kern = k_resident_mseq<float, L, NT>;
    const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (a != hipSuccess) return a;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or);
    return hipGetLastError();
}

hipError_t launch_resident_pair(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    if (e.precision == HSG_FP64) return dispatch_pair<double>(e, n_sweeps, n_hb, n_or, st);
    return dispatch_pair<float>(e, n_sweeps, n_hb, n_or, st);
}

hipError_t launch_resident(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                           int parity, int block_threads, hipStream_t st) {
    (void)default_threads;
    if (e.precision == HSG_FP64)
        return dispatch<double>(e, n_sweeps, n_hb, n_or, anneal, parity, block_threads, st);
    return dispatch<float>(e, n_sweeps, n_hb, n_or, anneal, parity, block_threads, st);
}

}  // namespace hsg
