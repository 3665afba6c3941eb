// Wavefront sweeps for lattices whose replica does not fit one workgroup's LDS
// (L = 18 .. 40 in binary32, .. 28 in binary64).
//
// One workgroup owns one replica and walks its z-planes.  A lattice sweep updates
// every site of parity 0 (W) and then every site of parity 1 (B); a W site of plane
// k needs the old B spins of planes k-1, k, k+1 and a B site of plane k the new W
// spins of planes k-1, k, k+1.  So at step k the workgroup updates the W sites of
// plane k and then the B sites of plane k-1, whose W neighbours are all new by then,
// and plane k-1 is finished.  The periodic boundary closes the wave: the B sites of
// planes 0 and L-1 wait for the end (they need the new W spins of planes L-1 and 0),
// so planes 0, 1 and L-1 stay in LDS for the whole sweep while planes 2 .. L-2 pass
// through a ring of four.  Every site sees exactly the neighbours of the two-phase
// checkerboard sweep, so the result is that of the other sweep kernels bit for bit
// (same site arithmetic, same random numbers); HBM sees one read and one write of
// the replica per lattice sweep instead of per half-sweep.  Each step is a handful of
// barrier-separated plane updates of one replica, so the walk is latency-bound: at
// L = 20 .. 40 it runs at 50-90 site updates per ns against 110 for the streaming
// kernels, which is why it is a tuning option (path 4) and not the default.
#include "hsg_device.h"
#include "hsg_launch.h"

namespace hsg {

template <int L>
__device__ __forceinline__ int wave_slot(int k) {
    return k == 0 ? 0 : (k == 1 ? 1 : (k == L - 1 ? 2 : 3 + (k & 3)));
}
constexpr int kWaveSlots = 7;

// plane k (both sublattices, three components: [mu][parity][L^2/2]) between the
// replica in global memory and its LDS slot
template <typename T, int L, int NT, bool STORE>
__device__ __forceinline__ void wave_copy(T* __restrict__ lds, T* __restrict__ g, int k) {
    constexpr int PL = L * L / 2, NH = L * L * L / 2;
    T* s = lds + wave_slot<L>(k) * 6 * PL;
    for (int v = static_cast<int>(threadIdx.x); v < 6 * PL; v += NT) {
        const int c = v / PL;  // mu * 2 + parity
        const int r = v - c * PL;
        T* gp = g + static_cast<size_t>(c) * NH + static_cast<size_t>(k) * PL + r;
        if (STORE)
            *gp = s[v];
        else
            s[v] = *gp;
    }
}

// Per-thread registers for the pipeline: one plane of spins in flight from HBM, and
// the six couplings of each of the thread's sites in a plane (MS sites per thread).
template <typename T, int L, int NT>
struct WavePlane {
    static constexpr int PL = L * L / 2, PV = (6 * PL + NT - 1) / NT;
    T v[PV];
};
template <typename T, int L, int NT>
struct WaveBonds {
    static constexpr int PL = L * L / 2, MS = (PL + NT - 1) / NT;
    T j[MS][6];
};

template <typename T, int L, int NT>
__device__ __forceinline__ void plane_fetch(WavePlane<T, L, NT>& r, const T* __restrict__ g, int k) {
    constexpr int PL = L * L / 2, NH = L * L * L / 2;
#pragma unroll
    for (int i = 0; i < WavePlane<T, L, NT>::PV; ++i) {
        const int v = static_cast<int>(threadIdx.x) + i * NT;
        const int c = v / PL;
        if (v < 6 * PL) r.v[i] = g[static_cast<size_t>(c) * NH + static_cast<size_t>(k) * PL + (v - c * PL)];
    }
}

template <typename T, int L, int NT>
__device__ __forceinline__ void plane_put(const WavePlane<T, L, NT>& r, T* __restrict__ lds, int k) {
    constexpr int PL = L * L / 2;
    T* s = lds + wave_slot<L>(k) * 6 * PL;
#pragma unroll
    for (int i = 0; i < WavePlane<T, L, NT>::PV; ++i) {
        const int v = static_cast<int>(threadIdx.x) + i * NT;
        if (v < 6 * PL) s[v] = r.v[i];
    }
}

// in-plane neighbour indices of site q (parity P, plane k): +x, -x, +y, -y, +z, -z
template <int L>
__device__ __forceinline__ void wave_nbrs(int q, int P, int k, int* nq) {
    constexpr int HL = L / 2;
    const int ih = q % HL, j = q / HL;
    const int o = (P + j + k) & 1;  // x = 2 ih + o
    int ixp = ih + o;
    if (ixp == HL) ixp = 0;
    int ixm = ih - 1 + o;
    if (ixm < 0) ixm = HL - 1;
    const int jp = j == L - 1 ? 0 : j + 1, jm = j == 0 ? L - 1 : j - 1;
    nq[0] = j * HL + ixp;
    nq[1] = j * HL + ixm;
    nq[2] = jp * HL + ih;
    nq[3] = jm * HL + ih;
    nq[4] = q;
    nq[5] = q;
}

// the couplings of the thread's sites of parity P in plane k (bond to +mu stored at
// the site, to -mu at the -mu neighbour)
template <typename T, int L, int NT>
__device__ __forceinline__ void bonds_fetch(WaveBonds<T, L, NT>& b, const T* __restrict__ J, int P, int k) {
    constexpr int PL = L * L / 2, NH = PL * L;
    const int O = 1 - P, km = k == 0 ? L - 1 : k - 1;
#pragma unroll
    for (int m = 0; m < WaveBonds<T, L, NT>::MS; ++m) {
        const int q = static_cast<int>(threadIdx.x) + m * NT;
        if (q >= PL) break;
        int nq[6];
        wave_nbrs<L>(q, P, k, nq);
        const int h = k * PL + q;
        b.j[m][0] = J[(0 * 2 + P) * NH + h];
        b.j[m][1] = J[(0 * 2 + O) * NH + k * PL + nq[1]];
        b.j[m][2] = J[(1 * 2 + P) * NH + h];
        b.j[m][3] = J[(1 * 2 + O) * NH + k * PL + nq[3]];
        b.j[m][4] = J[(2 * 2 + P) * NH + h];
        b.j[m][5] = J[(2 * 2 + O) * NH + km * PL + q];
    }
}

// The sites of parity P in plane k, heat-bath (HB) or overrelaxation, all neighbours
// in LDS; the energy and norm check of the last half-sweep fused (want).
template <typename T, int L, int NT, bool HB>
__device__ __forceinline__ void wave_update(T* __restrict__ lds, const WaveBonds<T, L, NT>& b, int P, int k,
                                            int hs, T beta, uint32_t tsw, uint32_t g, uint32_t k0,
                                            uint32_t k1, bool want, bool rn, double& acc, bool& bad) {
    constexpr int HL = L / 2, PL = HL * L, NH = PL * L, NQ = NH / 2;
    const int km = k == 0 ? L - 1 : k - 1, kp = k == L - 1 ? 0 : k + 1;
    const int O = 1 - P;
    T* cur = lds + wave_slot<L>(k) * 6 * PL;
    const T* below = lds + wave_slot<L>(km) * 6 * PL;
    const T* above = lds + wave_slot<L>(kp) * 6 * PL;
    const uint32_t c3 = heatbath_c3(hs);
#pragma unroll
    for (int m = 0; m < WaveBonds<T, L, NT>::MS; ++m) {
        const int q = static_cast<int>(threadIdx.x) + m * NT;
        if (q >= PL) break;
        int nq[6];
        wave_nbrs<L>(q, P, k, nq);
        const int h = k * PL + q;
        const T* pl[6] = {cur, cur, cur, cur, above, below};
        T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const T* src = pl[d];
            Sx = fma(b.j[m][d], src[(0 * 2 + O) * PL + nq[d]], Sx);
            Sy = fma(b.j[m][d], src[(1 * 2 + O) * PL + nq[d]], Sy);
            Sz = fma(b.j[m][d], src[(2 * 2 + O) * PL + nq[d]], Sz);
        }
        T* w0 = cur + (0 * 2 + P) * PL;
        T* w1 = cur + (1 * 2 + P) * PL;
        T* w2 = cur + (2 * 2 + P) * PL;
        T ox, oy, oz;
        if constexpr (HB) {
            T r1, r2;
            if constexpr (sizeof(T) == 4) {  // one block per site pair (h, h + N/4)
                const bool hi = h >= NQ;
                const Words w = philox(static_cast<uint32_t>(hi ? h - NQ : h), tsw, g, c3, k0, k1);
                r1 = static_cast<T>(u01_23(hi ? w.w2 : w.w0));
                r2 = static_cast<T>(u01_23(hi ? w.w3 : w.w1));
            } else {
                const Words w = philox(static_cast<uint32_t>(h), tsw, g, c3, k0, k1);
                r1 = static_cast<T>(u01_52(w.w0, w.w1));
                r2 = static_cast<T>(u01_52(w.w2, w.w3));
            }
            heatbath<T>(Sx, Sy, Sz, beta, r1, r2, ox, oy, oz);
        } else {
            overrelax<T>(w0[q], w1[q], w2[q], Sx, Sy, Sz, ox, oy, oz);
            if (rn) renormalize(ox, oy, oz);
        }
        w0[q] = ox;
        w1[q] = oy;
        w2[q] = oz;
        if (want) {
            const double dx = ox, dy = oy, dz = oz;
            acc += fma(dz, static_cast<double>(Sz), fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
            const double n2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (!(fabs(n2 - 1.0) <= NormTol<T>::value)) bad = true;
        }
    }
}

template <typename T, int L, int NT>
__device__ __forceinline__ void wave_update_any(bool hb, T* lds, const WaveBonds<T, L, NT>& b, int P, int k,
                                                int hs, T beta, uint32_t tsw, uint32_t g, uint32_t k0,
                                                uint32_t k1, bool want, bool rn, double& acc, bool& bad) {
    if (hb)
        wave_update<T, L, NT, true>(lds, b, P, k, hs, beta, tsw, g, k0, k1, want, false, acc, bad);
    else
        wave_update<T, L, NT, false>(lds, b, P, k, hs, beta, tsw, g, k0, k1, want, rn, acc, bad);
}

// n_sweeps sweeps (n_hb heat-bath then n_or overrelaxation lattice sweeps each) of
// replica xcd_order(blockIdx.x) at its own temperature.  Inside a lattice sweep the
// barriers are LDS-only (lds_barrier), so the plane and coupling fetches issued at the
// top of a step stay in flight across them; the full barriers at its ends also order
// the global stores of one lattice sweep before the loads of the next.
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_wave(hsg_ensemble e, int n_sweeps, int n_hb, int n_or) {
    constexpr int N = L * L * L;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[(NT + 63) / 64];

    const int slot = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int C = e.n_chains, R = e.n_temps;
    const int smp = slot / (C * R);
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    T* gs = static_cast<T*>(e.spins) + static_cast<size_t>(slot) * 3 * N;
    const uint32_t g = e.slot_base + static_cast<uint32_t>(slot);
    const uint32_t t0 = e.sweep_ctr[slot];
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const T beta = static_cast<T>(e.betas[label(e.temp_of_slot[slot], R, e.guard)]);
    const int nlat = n_hb + n_or;
    double acc = 0.0;
    bool bad = false;
    WavePlane<T, L, NT> pf;                 // next ring plane, in flight
    WaveBonds<T, L, NT> bw, bb, bw_n, bb_n;  // couplings: W of plane k, B of plane k-1, and the next ones
    for (int s = 0; s < n_sweeps; ++s) {
        const uint32_t tsw = t0 + static_cast<uint32_t>(s);
        for (int l = 0; l < nlat; ++l) {
            const bool hb = l < n_hb;
            const bool rn = renorm_on(e) && n_hb == 0 && l == nlat - 1;  // renormalised once per sweep
            const bool want = (s == n_sweeps - 1) && (l == nlat - 1);
            const int hs0 = 2 * l, hs1 = 2 * l + 1;
            // planes L-1, 0, 1 and 2, and the couplings of the first two steps
            wave_copy<T, L, NT, false>(lds, gs, L - 1);
            wave_copy<T, L, NT, false>(lds, gs, 0);
            wave_copy<T, L, NT, false>(lds, gs, 1);
            wave_copy<T, L, NT, false>(lds, gs, 2);
            bonds_fetch<T, L, NT>(bw, J, 0, 0);
            bonds_fetch<T, L, NT>(bw_n, J, 0, 1);
            __syncthreads();
            wave_update_any<T, L, NT>(hb, lds, bw, 0, 0, hs0, beta, tsw, g, k0, k1, false, rn, acc, bad);
            lds_barrier();
            bw = bw_n;
            for (int k = 1; k < L; ++k) {
                // step k: W sites of plane k, then B sites of plane k-1.  Plane k+1
                // arrived during step k-1; plane k+2 and the couplings of step k+1 are
                // fetched now and arrive during this step's arithmetic.
                if (k + 1 >= 3 && k + 1 <= L - 2) plane_put<T, L, NT>(pf, lds, k + 1);
                if (k + 2 >= 3 && k + 2 <= L - 2) plane_fetch<T, L, NT>(pf, gs, k + 2);
                if (k + 1 <= L - 1) bonds_fetch<T, L, NT>(bw_n, J, 0, k + 1);
                if (k - 1 >= 1) {
                    if (k == 2) bonds_fetch<T, L, NT>(bb, J, 1, 1);
                    bonds_fetch<T, L, NT>(bb_n, J, 1, k);
                }
                lds_barrier();
                wave_update_any<T, L, NT>(hb, lds, bw, 0, k, hs0, beta, tsw, g, k0, k1, false, rn, acc, bad);
                lds_barrier();
                if (k - 1 >= 1) {
                    wave_update_any<T, L, NT>(hb, lds, bb, 1, k - 1, hs1, beta, tsw, g, k0, k1, want, rn, acc, bad);
                    lds_barrier();
                    wave_copy<T, L, NT, true>(lds, gs, k - 1);
                    bb = bb_n;
                }
                bw = bw_n;
            }
            // B sites of planes L-1 (couplings fetched at step L-1) and 0
            bonds_fetch<T, L, NT>(bw_n, J, 1, 0);
            wave_update_any<T, L, NT>(hb, lds, bb, 1, L - 1, hs1, beta, tsw, g, k0, k1, want, rn, acc, bad);
            wave_update_any<T, L, NT>(hb, lds, bw_n, 1, 0, hs1, beta, tsw, g, k0, k1, want, rn, acc, bad);
            lds_barrier();
            wave_copy<T, L, NT, true>(lds, gs, L - 1);
            wave_copy<T, L, NT, true>(lds, gs, 0);
            __syncthreads();  // the next lattice sweep reloads these planes
        }
    }
    const double tot = block_sum<NT>(acc, red);
    if (bad || !isfinite(tot)) atomicOr(e.guard, 1);
    if (threadIdx.x == 0) {
        if (n_sweeps > 0) e.energy[slot] = -tot;
        e.sweep_ctr[slot] = t0 + static_cast<uint32_t>(n_sweeps);
    }
}

template <typename T, int L>
static hipError_t go_wave(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    constexpr int PL = L * L / 2;
    constexpr int NT = PL >= 512 ? 512 : ((PL + 63) / 64) * 64;
    constexpr size_t lds = static_cast<size_t>(kWaveSlots) * 6 * PL * sizeof(T);
    auto kern = k_wave<T, L, NT>;
    const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (a != hipSuccess) return a;
    const int blocks = e.n_samples * e.n_chains * e.n_temps;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, n_sweeps, n_hb, n_or);
    return hipGetLastError();
}

template <typename T>
static hipError_t wave_dispatch(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    switch (e.L) {
        case 18: return go_wave<T, 18>(e, n_sweeps, n_hb, n_or, st);
        case 20: return go_wave<T, 20>(e, n_sweeps, n_hb, n_or, st);
        case 22: return go_wave<T, 22>(e, n_sweeps, n_hb, n_or, st);
        case 24: return go_wave<T, 24>(e, n_sweeps, n_hb, n_or, st);
        case 26: return go_wave<T, 26>(e, n_sweeps, n_hb, n_or, st);
        case 28: return go_wave<T, 28>(e, n_sweeps, n_hb, n_or, st);
        case 30:
            if constexpr (sizeof(T) == 4) return go_wave<T, 30>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        case 32:
            if constexpr (sizeof(T) == 4) return go_wave<T, 32>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        case 34:
            if constexpr (sizeof(T) == 4) return go_wave<T, 34>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        case 36:
            if constexpr (sizeof(T) == 4) return go_wave<T, 36>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        case 38:
            if constexpr (sizeof(T) == 4) return go_wave<T, 38>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        case 40:
            if constexpr (sizeof(T) == 4) return go_wave<T, 40>(e, n_sweeps, n_hb, n_or, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

bool wave_supported(const hsg_ensemble& e) {
    if (e.L < 18 || e.L > 40 || (e.L & 1)) return false;
    const size_t t = e.precision == HSG_FP64 ? 8 : 4;
    const size_t lds = static_cast<size_t>(kWaveSlots) * 6 * (static_cast<size_t>(e.L) * e.L / 2) * t;
    if (e.precision == HSG_FP64 && e.L > 28) return false;
    return lds <= max_block_lds();
}

hipError_t launch_wave_sweeps(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st) {
    if (e.precision == HSG_FP64) return wave_dispatch<double>(e, n_sweeps, n_hb, n_or, st);
    return wave_dispatch<float>(e, n_sweeps, n_hb, n_or, st);
}

}  // namespace hsg
