// Initialisation, energy, replica-exchange and measurement kernels.
#include "hsg_device.h"
#include "hsg_launch.h"

namespace hsg {

// ---------------------------------------------------------------- initialisation
// J(x, mu) ~ N(0,1) (paper Sec. I), Box-Muller cosine branch in FP64 from two
// 52-bit uniforms of the block (x, mu, sample, 1<<24); stored at [s][mu][p(x)][h(x)].
template <typename T>
__global__ void k_init_couplings(hsg_ensemble e) {
    const int L = e.L;
    const int N = L * L * L, NH = N / 2;
    const size_t total = static_cast<size_t>(e.n_samples) * N * 3;
    const size_t id = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int mu = static_cast<int>(id % 3);
    const int x = static_cast<int>((id / 3) % N);
    const int s = static_cast<int>(id / (3 * static_cast<size_t>(N)));
    const Words w = philox(static_cast<uint32_t>(x), static_cast<uint32_t>(mu), e.sample_base + s,
                           kTagCoupling << 24, key_lo(e.seed), key_hi(e.seed));
    const double r1 = u01_52(w.w0, w.w1), r2 = u01_52(w.w2, w.w3);
    const double gval = sqrt(-2.0 * log(r1)) * cos(2.0 * 3.14159265358979323846 * r2);
    const int i = x % L, row = x / L, j = row % L, k = row / L;
    const int p = (i + j + k) & 1;
    const int h = i / 2 + (L / 2) * row;
    T* J = static_cast<T*>(e.couplings) + static_cast<size_t>(s) * 3 * N;
    J[(mu * 2 + p) * NH + h] = static_cast<T>(gval);
}

// Uniform unit spins: z = 2 r1 - 1, azimuth 2 pi r2 (block (x, 0, slot, 2<<24));
// cold start (1, 0, 0).
template <typename T>
__global__ void k_init_spins(hsg_ensemble e, int cold) {
    const int L = e.L;
    const int N = L * L * L, NH = N / 2;
    const size_t n_slots = static_cast<size_t>(e.n_samples) * e.n_chains * e.n_temps;
    const size_t id = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= n_slots * N) return;
    const int x = static_cast<int>(id % N);
    const size_t slot = id / N;
    double v0 = 1.0, v1 = 0.0, v2 = 0.0;
    if (!cold) {
        const Words w = philox(static_cast<uint32_t>(x), 0u, e.slot_base + static_cast<uint32_t>(slot),
                               kTagInit << 24, key_lo(e.seed), key_hi(e.seed));
        const double r1 = u01_52(w.w0, w.w1), r2 = u01_52(w.w2, w.w3);
        const double z = 2.0 * r1 - 1.0;
        const double rho = 2.0 * sqrt(r1 * (1.0 - r1));
        const double phi = 2.0 * 3.14159265358979323846 * r2;
        v0 = rho * cos(phi);
        v1 = rho * sin(phi);
        v2 = z;
    }
    const int i = x % L, row = x / L, j = row % L, k = row / L;
    const int p = (i + j + k) & 1;
    const int h = i / 2 + (L / 2) * row;
    T* s = static_cast<T*>(e.spins) + slot * 3 * N;
    s[(0 * 2 + p) * NH + h] = static_cast<T>(v0);
    s[(1 * 2 + p) * NH + h] = static_cast<T>(v1);
    s[(2 * 2 + p) * NH + h] = static_cast<T>(v2);
}

__global__ void k_reset_state(hsg_ensemble e) {
    const int R = e.n_temps;
    const int n_chains = e.n_samples * e.n_chains;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id == 0) *e.guard = 0;
    if (id >= n_chains * R) return;
    const int r = id % R, ch = id / R;
    e.temp_of_slot[id] = r;
    e.slot_of_temp[id] = r;
    e.sweep_ctr[id] = 0u;
    e.rt_state[id] = r == 0 ? 1 : 0;
    e.rt_trips[id] = 0;
    if (r < R - 1) {
        e.swap_stats[(static_cast<size_t>(ch) * (R - 1) + r) * 2] = 0;
        e.swap_stats[(static_cast<size_t>(ch) * (R - 1) + r) * 2 + 1] = 0;
    }
    if (r == 0) e.swap_ctr[ch] = 0u;
}

// ---------------------------------------------------------------- energy
// H = -sum_{x in W} s_x . S_x in FP64 (equal to the bond sum of Eq. (2): every
// bond has exactly one white end).  One workgroup per slot.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_energy(hsg_ensemble e, double* out) {
    __shared__ double red[NT / 64];
    const int L = e.L;
    const int N = L * L * L, NH = N / 2;
    const int slot = blockIdx.x;
    const int C = e.n_chains, R = e.n_temps;
    const int smp = slot / (C * R);
    const T* s = static_cast<const T*>(e.spins) + static_cast<size_t>(slot) * 3 * N;
    const T* J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    double acc = 0.0;
    for (int h = threadIdx.x; h < NH; h += NT) {
        const Nbr nb = neighbours<0>(h, 0, L);
        double S[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const double jp = J[(mu * 2 + 0) * NH + h];
            const double jm = J[(mu * 2 + 1) * NH + nb.n[2 * mu + 1]];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S[a] += jp * static_cast<double>(s[(a * 2 + 1) * NH + nb.n[2 * mu]]);
                S[a] += jm * static_cast<double>(s[(a * 2 + 1) * NH + nb.n[2 * mu + 1]]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) acc += static_cast<double>(s[(a * 2 + 0) * NH + h]) * S[a];
    }
    const double tot = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) {
        const double H = -tot;
        if (!isfinite(H)) atomicOr(e.guard, 1);
        if (out)
            out[slot] = H;
        else
            e.energy[slot] = H;
    }
}

// ---------------------------------------------------------------- exchange
__device__ __forceinline__ void roundtrip_update(int R, const int* tos, int* st, long long* trips) {
    for (int r = 0; r < R; ++r) {
        const int T = tos[r];  // range-checked by the caller's labels
        if (T == 0) {
            if (st[r] == 2) trips[r] += 1;
            st[r] = 1;
        } else if (T == R - 1) {
            if (st[r] == 1) st[r] = 2;
        }
    }
}

// x = sot[i], y = sot[i + 1] (already range-checked by the caller)
__device__ __forceinline__ void relabel(int* tos, int* sot, int i, int x, int y) {
    sot[i] = y;
    sot[i + 1] = x;
    tos[x] = i + 1;
    tos[y] = i;
}

__device__ __forceinline__ double swap_uniform(const hsg_ensemble& e, int i, uint32_t n, uint32_t cg) {
    const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, key_lo(e.seed), key_hi(e.seed));
    return u01_52(w.w0, w.w1);
}

// Eq. (1): accept iff ln u < (beta_{i+1} - beta_i)(H_{i+1} - H_i).  One wave per
// chain: labels and energies are staged in LDS and every pair's uniform and its
// logarithm are computed in parallel.  Even or odd pairs are disjoint: each lane
// decides its own.  In ascending order pair i sees at temperature i the
// configuration the previous pair left there (the "carry": the one it moved up, or
// the one it kept), and at i + 1 the configuration that was there before the pass;
// so the per-pair inputs (ln u, the beta step, the upper configuration and its
// energy) are all staged in parallel and one lane runs the carry through the pairs
// with no load that depends on an earlier decision.  The wave then writes labels,
// statistics and round-trip state back in parallel.
constexpr int kSwapMaxR = 256;

__global__ void __launch_bounds__(64) k_swap(hsg_ensemble e, int pairing) {
    __shared__ int s_sot[kSwapMaxR], s_tos[kSwapMaxR], s_up[kSwapMaxR];
    __shared__ double s_en[kSwapMaxR], s_lu[kSwapMaxR], s_db[kSwapMaxR], s_eup[kSwapMaxR];
    __shared__ unsigned char s_acc[kSwapMaxR];
    const int ch = blockIdx.x;
    const int lane = threadIdx.x;
    const int R = e.n_temps;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    const double* en = e.energy + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    for (int r = lane; r < R; r += 64) {
        s_sot[r] = label(sot[r], R, e.guard);
        s_en[r] = en[r];
    }
    for (int i = lane; i < R - 1; i += 64) {
        const bool sel = pairing == 0 || (pairing == 1 && !(i & 1)) || (pairing == 2 && (i & 1));
        s_lu[i] = sel ? log(swap_uniform(e, i, n, cg)) : 0.0;
        s_db[i] = e.betas[i + 1] - e.betas[i];
        s_acc[i] = sel ? 2 : 0;  // 2 = attempted, 3 = accepted
    }
    __syncthreads();
    if (pairing == 0) {
        for (int i = lane; i < R - 1; i += 64) {  // the configuration above pair i before the pass
            s_up[i] = s_sot[i + 1];
            s_eup[i] = s_en[s_sot[i + 1]];
        }
        __syncthreads();
        if (lane == 0) {
            int carry = s_sot[0];
            double ec = s_en[carry];
            for (int i = 0; i < R - 1; ++i) {
                const int y = s_up[i];
                const double ey = s_eup[i];
                const bool ok = s_lu[i] < s_db[i] * (ey - ec);
                s_sot[i] = ok ? y : carry;
                s_acc[i] = ok ? 3 : 2;
                if (!ok) {
                    carry = y;
                    ec = ey;
                }
            }
            s_sot[R - 1] = carry;
        }
    } else {
        for (int i = lane; i < R - 1; i += 64) {  // disjoint pairs
            if (!s_acc[i]) continue;
            const int x = s_sot[i], y = s_sot[i + 1];
            if (s_lu[i] < s_db[i] * (s_en[y] - s_en[x])) {
                s_sot[i] = y;
                s_sot[i + 1] = x;
                s_acc[i] = 3;
            }
        }
    }
    __syncthreads();
    for (int t = lane; t < R; t += 64) {
        sot[t] = s_sot[t];
        s_tos[s_sot[t]] = t;
    }
    for (int i = lane; i < R - 1; i += 64) {
        if (s_acc[i]) {
            st[2 * i] += 1;
            if (s_acc[i] == 3) st[2 * i + 1] += 1;
        }
    }
    __syncthreads();
    int* rs = e.rt_state + static_cast<size_t>(ch) * R;
    long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + static_cast<size_t>(ch) * R;
    for (int r = lane; r < R; r += 64) {
        const int T = s_tos[r];
        tos[r] = T;
        if (T == 0) {
            if (rs[r] == 2) rtt[r] += 1;
            rs[r] = 1;
        } else if (T == R - 1) {
            if (rs[r] == 1) rs[r] = 2;
        }
    }
    if (lane == 0) e.swap_ctr[ch] = n + 1u;
}

// The same exchange for ladders of at most 64 temperatures, one wave per chain with
// lane r holding temperature r's label, slot r's energy and its round-trip state, and
// pair r's statistics.  Nothing it loads depends on a decision, so every load is issued
// at entry and the kernel makes one trip to memory instead of three; labels and
// energies move between lanes by cross-lane permutes, and the ascending pass reads each
// pair's inputs from the lane that holds them.  Decisions, labels, statistics and round
// trips are those of k_swap bit for bit (the same operations on the same values).
constexpr int kSwapWaveMaxR = 64;

__global__ void __launch_bounds__(64) k_swap_wave(hsg_ensemble e, int pairing) {
    const int ch = blockIdx.x;
    const int lane = threadIdx.x;
    const int R = e.n_temps;
    const bool tl = lane < R, pl = lane < R - 1;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    const double* en = e.energy + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    int* rs = e.rt_state + static_cast<size_t>(ch) * R;
    long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + static_cast<size_t>(ch) * R;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    int x = tl ? sot[lane] : lane;
    const double e_slot = tl ? en[lane] : 0.0;
    const double b0 = pl ? e.betas[lane] : 0.0, b1 = pl ? e.betas[lane + 1] : 0.0;
    const long long n_att = pl ? st[2 * lane] : 0, n_acc = pl ? st[2 * lane + 1] : 0;
    const int rs_old = tl ? rs[lane] : 0;
    const long long trips = tl ? rtt[lane] : 0;
    if (tl) x = label(x, R, e.guard);
    const bool sel = pl && (pairing == 0 || (pairing == 1 && !(lane & 1)) || (pairing == 2 && (lane & 1)));
    const double lu = sel ? log(swap_uniform(e, lane, n, cg)) : 0.0;
    const double db = b1 - b0;
    const double ex = __shfl(e_slot, x);  // energy of the configuration at temperature lane
    const int up = __shfl_down(x, 1);      // the configuration above pair lane, before the pass
    const double eup = __shfl_down(ex, 1);
    int nx = x;
    int acc = sel ? 2 : 0;  // 2 = attempted, 3 = accepted
    if (pairing == 0) {
        int carry = __builtin_amdgcn_readlane(x, 0);
        double ec = readlane_f64(ex, 0);
        for (int i = 0; i < R - 1; ++i) {
            const int y = __builtin_amdgcn_readlane(up, i);
            const double ey = readlane_f64(eup, i);
            const bool ok = readlane_f64(lu, i) < readlane_f64(db, i) * (ey - ec);
            if (lane == i) {
                nx = ok ? y : carry;
                acc = ok ? 3 : 2;
            }
            if (!ok) {
                carry = y;
                ec = ey;
            }
        }
        if (lane == R - 1) nx = carry;
    } else {
        const bool ok = sel && lu < db * (eup - ex);
        const int below = __shfl_up(x, 1);
        const bool ok_below = __shfl_up(static_cast<int>(ok), 1) != 0 && lane > 0;
        if (ok) {
            nx = up;
            acc = 3;
        } else if (ok_below) {
            nx = below;
        }
    }
    // temperature of every slot: lane nx receives lane (lanes >= R map to themselves)
    const int T = __builtin_amdgcn_ds_permute(nx << 2, lane);
    if (tl) {
        sot[lane] = nx;
        tos[lane] = T;
        if (T == 0) {
            if (rs_old == 2) rtt[lane] = trips + 1;
            rs[lane] = 1;
        } else if (T == R - 1) {
            if (rs_old == 1) rs[lane] = 2;
        }
    }
    if (acc) {
        st[2 * lane] = n_att + 1;
        if (acc == 3) st[2 * lane + 1] = n_acc + 1;
    }
    if (lane == 0) e.swap_ctr[ch] = n + 1u;
}

// Annealed exchange decision: accept iff ln u < -(W_up + W_dn); the annealed
// states (candidate buffer) replace the accepted slots, energies follow.
__global__ void k_anneal_decide(hsg_ensemble e, int parity) {
    const int n_chains = e.n_samples * e.n_chains;
    const int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= n_chains) return;
    const int R = e.n_temps;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const double* cen = reinterpret_cast<const double*>(scr + sl.cand_energy);
    int* flags = reinterpret_cast<int*>(scr + sl.flags);
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    double* en = e.energy + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const double* W = e.work + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    for (int r = 0; r < R; ++r) flags[ch * R + r] = 0;
    for (int i = parity; i < R - 1; i += 2) {
        const int x = label(sot[i], R, e.guard), y = label(sot[i + 1], R, e.guard);
        int K = e.anneal_K[i];
        K = K < 0 ? 0 : (K > e.anneal_K_max ? e.anneal_K_max : K);
        const double wsum = W[2 * i] + W[2 * i + 1];
        const double u = swap_uniform(e, i, n, cg);
        st[2 * i] += 1;
        if (log(u) < -wsum) {
            en[x] = cen[ch * R + x];
            en[y] = cen[ch * R + y];
            if (K > 0) {
                flags[ch * R + x] = 1;
                flags[ch * R + y] = 1;
            }
            relabel(tos, sot, i, x, y);
            st[2 * i + 1] += 1;
        }
    }
    e.swap_ctr[ch] = n + 1u;
    roundtrip_update(R, tos, e.rt_state + static_cast<size_t>(ch) * R,
                     reinterpret_cast<long long*>(e.rt_trips) + static_cast<size_t>(ch) * R);
}

template <typename T>
__global__ void k_anneal_copyback(hsg_ensemble e) {
    const int slot = blockIdx.x;
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const int* flags = reinterpret_cast<const int*>(scr + sl.flags);
    if (!flags[slot]) return;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const T*>(scr + sl.cand) + slot * 3 * N);
    uint4* dst = reinterpret_cast<uint4*>(static_cast<T*>(e.spins) + slot * 3 * N);
    const size_t nv = 3 * N * sizeof(T) / 16;
    for (size_t v = threadIdx.x; v < nv; v += blockDim.x) dst[v] = src[v];
}

// ---------------------------------------------------------------- measurement
// Q_ab = sum_x s^(0)_{a,x} s^(1)_{b,x} between chains 0 and 1 at temperature b,
// chi = Q:Q / N (paper Sec. II); e = H/N by temperature.  Workgroup per (sample, b).
// FIN: first finish a streaming sweep whose last finishing pass was left out: the
// energy of each slot it reads from the per-tile sums (n_tiles of them, added in tile
// order, as k_stream_finalize adds them), and sweep_ctr += ctr_add.  Every slot is one
// (sample, chain, temperature), so each is finished by exactly one workgroup.
template <typename T, int NT, bool FIN = false>
__global__ void __launch_bounds__(NT) k_measure(hsg_ensemble e, int n_tiles = 0, int ctr_add = 0) {
    constexpr int NW = NT / 64;
    __shared__ double red[9 * NW];
    const int N = e.L * e.L * e.L;
    const int R = e.n_temps, C = e.n_chains;
    const int smp = blockIdx.x / R, b = blockIdx.x % R;
    if (FIN) {
        // one wave per chain: its lanes load 64 per-tile sums at a time, which are then
        // added one lane after another (the finishing pass's order)
        const ScratchLayout sl = scratch_layout(e);
        const double* part = reinterpret_cast<const double*>(static_cast<const unsigned char*>(e.scratch) + sl.partial);
        const int lane = threadIdx.x & 63;
        for (int c = threadIdx.x >> 6; c < C; c += NW) {
            const int slot = (smp * C + c) * R + label(e.slot_of_temp[(smp * C + c) * R + b], R, e.guard);
            const double* ps = part + static_cast<size_t>(slot) * sl.max_tiles;
            double H = 0.0;
            for (int t0 = 0; t0 < n_tiles; t0 += 64) {
                const double v = t0 + lane < n_tiles ? ps[t0 + lane] : 0.0;
                const int m = n_tiles - t0 < 64 ? n_tiles - t0 : 64;
                for (int j = 0; j < m; ++j) H += readlane_f64(v, j);
            }
            if (lane == 0) {
                if (!isfinite(H)) atomicOr(e.guard, 1);
                e.energy[slot] = H;
                e.sweep_ctr[slot] += static_cast<uint32_t>(ctr_add);
                e.e_temp[(static_cast<size_t>(smp) * C + c) * R + b] = H / static_cast<double>(N);
            }
        }
    } else {
        for (int c = threadIdx.x; c < C; c += NT) {
            const int slot = (smp * C + c) * R + label(e.slot_of_temp[(smp * C + c) * R + b], R, e.guard);
            e.e_temp[(static_cast<size_t>(smp) * C + c) * R + b] = e.energy[slot] / static_cast<double>(N);
        }
    }
    if (C < 2 || e.Q == nullptr) return;  // uniform over the block
    const int s1 = (smp * C + 0) * R + label(e.slot_of_temp[(smp * C + 0) * R + b], R, e.guard);
    const int s2 = (smp * C + 1) * R + label(e.slot_of_temp[(smp * C + 1) * R + b], R, e.guard);
    // 16-byte loads of W consecutive sites of a component (N is a multiple of 8 and
    // every replica starts on a 16-byte boundary)
    constexpr int W = 16 / static_cast<int>(sizeof(T));
    struct alignas(16) Vec { T v[W]; };
    const int NV = N / W;
    const Vec* a = reinterpret_cast<const Vec*>(static_cast<const T*>(e.spins) + static_cast<size_t>(s1) * 3 * N);
    const Vec* c = reinterpret_cast<const Vec*>(static_cast<const T*>(e.spins) + static_cast<size_t>(s2) * 3 * N);
    double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4  // all loads of a 16^3 replica pair issued before the first use
    for (int v = threadIdx.x; v < NV; v += NT) {
        const Vec a0 = a[v], a1 = a[NV + v], a2 = a[2 * NV + v];
        const Vec c0 = c[v], c1 = c[NV + v], c2 = c[2 * NV + v];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double x0 = a0.v[w], x1 = a1.v[w], x2 = a2.v[w];
            const double y0 = c0.v[w], y1 = c1.v[w], y2 = c2.v[w];
            q[0] = fma(x0, y0, q[0]); q[1] = fma(x0, y1, q[1]); q[2] = fma(x0, y2, q[2]);
            q[3] = fma(x1, y0, q[3]); q[4] = fma(x1, y1, q[4]); q[5] = fma(x1, y2, q[5]);
            q[6] = fma(x2, y0, q[6]); q[7] = fma(x2, y1, q[7]); q[8] = fma(x2, y2, q[8]);
        }
    }
    // nine sums at once: butterfly in each wave, then the waves in order
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double w = wave_sum(q[k]);
        if ((threadIdx.x & 63) == 0) red[k * NW + (threadIdx.x >> 6)] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double chi = 0.0;
        for (int k = 0; k < 9; ++k) {
            double t = 0.0;
            for (int w = 0; w < NW; ++w) t += red[k * NW + w];
            e.Q[(static_cast<size_t>(smp) * R + b) * 9 + k] = t;
            chi += t * t;
        }
        e.chi[static_cast<size_t>(smp) * R + b] = chi / static_cast<double>(N);
    }
}

// ---------------------------------------------------------------- launchers
static unsigned nblk(size_t n, unsigned t) { return static_cast<unsigned>((n + t - 1) / t); }

hipError_t launch_init_couplings(const hsg_ensemble& e, hipStream_t st) {
    const size_t total = static_cast<size_t>(e.n_samples) * e.L * e.L * e.L * 3;
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_init_couplings<double>, dim3(nblk(total, 256)), dim3(256), 0, st, e);
    else
        hipLaunchKernelGGL(k_init_couplings<float>, dim3(nblk(total, 256)), dim3(256), 0, st, e);
    return hipGetLastError();
}

hipError_t launch_init_spins(const hsg_ensemble& e, int cold, hipStream_t st) {
    const size_t n_slots = static_cast<size_t>(e.n_samples) * e.n_chains * e.n_temps;
    const size_t total = n_slots * e.L * e.L * e.L;
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_init_spins<double>, dim3(nblk(total, 256)), dim3(256), 0, st, e, cold);
    else
        hipLaunchKernelGGL(k_init_spins<float>, dim3(nblk(total, 256)), dim3(256), 0, st, e, cold);
    hipLaunchKernelGGL(k_reset_state, dim3(nblk(n_slots, 256)), dim3(256), 0, st, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return launch_energy(e, nullptr, st);
}

hipError_t launch_energy(const hsg_ensemble& e, double* out, hipStream_t st) {
    const int n_slots = e.n_samples * e.n_chains * e.n_temps;
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL((k_energy<double, 256>), dim3(n_slots), dim3(256), 0, st, e, out);
    else
        hipLaunchKernelGGL((k_energy<float, 256>), dim3(n_slots), dim3(256), 0, st, e, out);
    return hipGetLastError();
}

hipError_t launch_swap(const hsg_ensemble& e, int pairing, hipStream_t st) {
    const int n_chains = e.n_samples * e.n_chains;
    if (e.n_temps > kSwapMaxR) return hipErrorInvalidValue;
    if (e.n_temps <= kSwapWaveMaxR)
        hipLaunchKernelGGL(k_swap_wave, dim3(n_chains), dim3(64), 0, st, e, pairing);
    else
        hipLaunchKernelGGL(k_swap, dim3(n_chains), dim3(64), 0, st, e, pairing);
    return hipGetLastError();
}

hipError_t launch_anneal_decide(const hsg_ensemble& e, int parity, hipStream_t st) {
    const int n_chains = e.n_samples * e.n_chains;
    const int n_slots = n_chains * e.n_temps;
    hipLaunchKernelGGL(k_anneal_decide, dim3(nblk(n_chains, 64)), dim3(64), 0, st, e, parity);
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_anneal_copyback<double>, dim3(n_slots), dim3(256), 0, st, e);
    else
        hipLaunchKernelGGL(k_anneal_copyback<float>, dim3(n_slots), dim3(256), 0, st, e);
    return hipGetLastError();
}

// Threads per measurement workgroup beyond L = 16.  The workgroups, one per (sample,
// temperature), are then few (8 x 32 at L = 32) and each streams a replica pair of
// 0.3-0.8 MB, so a workgroup needs many waves to keep enough loads in flight.  The
// size depends on L alone, so a sample range measured on its own sums in the same order.
constexpr int kMeasureThreadsLarge = 512;

hipError_t launch_measure(const hsg_ensemble& e, hipStream_t st) {
    const int blocks = e.n_samples * e.n_temps;
    if (e.L > 16) {
        constexpr int NT = kMeasureThreadsLarge;
        if (e.precision == HSG_FP64)
            hipLaunchKernelGGL((k_measure<double, NT>), dim3(blocks), dim3(NT), 0, st, e, 0, 0);
        else
            hipLaunchKernelGGL((k_measure<float, NT>), dim3(blocks), dim3(NT), 0, st, e, 0, 0);
        return hipGetLastError();
    }
    // one (sample, temperature) per 128-thread workgroup: 1536 of them at L = 16, 64 x 24
    // (measured 26.4 us per pass against 27.3 with 256 threads and 28.1 with 512)
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL((k_measure<double, 128>), dim3(blocks), dim3(128), 0, st, e, 0, 0);
    else
        hipLaunchKernelGGL((k_measure<float, 128>), dim3(blocks), dim3(128), 0, st, e, 0, 0);
    return hipGetLastError();
}

hipError_t launch_measure_fin(const hsg_ensemble& e, int n_tiles, int ctr_add, hipStream_t st) {
    const int blocks = e.n_samples * e.n_temps;
    if (e.L > 16) {
        constexpr int NT = kMeasureThreadsLarge;
        if (e.precision == HSG_FP64)
            hipLaunchKernelGGL((k_measure<double, NT, true>), dim3(blocks), dim3(NT), 0, st, e, n_tiles, ctr_add);
        else
            hipLaunchKernelGGL((k_measure<float, NT, true>), dim3(blocks), dim3(NT), 0, st, e, n_tiles, ctr_add);
    } else {
        if (e.precision == HSG_FP64)
            hipLaunchKernelGGL((k_measure<double, 128, true>), dim3(blocks), dim3(128), 0, st, e, n_tiles, ctr_add);
        else
            hipLaunchKernelGGL((k_measure<float, 128, true>), dim3(blocks), dim3(128), 0, st, e, n_tiles, ctr_add);
    }
    return hipGetLastError();
}

}  // namespace hsg
