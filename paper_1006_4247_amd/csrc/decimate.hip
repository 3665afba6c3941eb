// Decimated replica exchange (paper Sec. III.A).
//
// The spins of one sublattice D do not interact, so integrating them out of
// exp(-beta H) leaves one factor I(beta S_z) = 4 pi sinh(R_z)/R_z per z in D
// (Eq. (HI)), R_z = beta |S_z| with S_z the local field of the kept sublattice.
// Exchanging the kept fields of x (at beta_1) and y (at beta_2) is accepted with
// Eq. (eq:aswap),
//     ln A = sum_{z in D} h(b2 a_z) - h(b1 a_z) + h(b1 c_z) - h(b2 c_z),
// h(u) = ln(sinh(u)/u), a_z = |S_z(x)|, c_z = |S_z(y)| (the 4 pi and 1/R factors
// cancel).  An accepted pair exchanges temperature labels and draws the D spins
// of both configurations anew by heat-bath at their new temperatures; a
// rejected pair changes nothing.  The first pair decimates a random sublattice
// d_0 and the role alternates along the ladder, D_i = (d_0 + i) mod 2.
//
// Ascending order over all pairs (pairing 0) is sequential within a chain: one
// workgroup per chain walks the pairs.  The even or odd pairs (pairing 1, 2) are
// disjoint: one workgroup per pair.  Fields and ln A terms are per site, ln A and
// the energies are deterministic FP64 block sums; one lane decides.
#include "hsg_device.h"
#include <type_traits>

#include "hsg_launch.h"

namespace hsg {

constexpr uint32_t kTagDecimate = 5u;      // heat-bath re-insertion draws
constexpr uint32_t kTagDecimateRole = 6u;  // sublattice of the first pair
constexpr int kDecThreads = 256;

// h(u) = ln(sinh(u)/u) = u + ln((1 - e^{-2u})/(2u)), finite for all u >= 0.
__device__ __forceinline__ double log_sinhc(double u) {
    if (!(u > 0.0)) return 0.0;
    return u + log(-expm1(-2.0 * u) / (2.0 * u));
}

// Binary32 form of a site's ln[rho(a) / rho(c)], rho(s) = expm1(-2 b2 s) / expm1(-2 b1 s)
// (see the LDS-resident kernel; binary32 configurations): expm1(x),
// x <= 0, by its Taylor series for x > -1, else e^x - 1 from the hardware exp2
// (e^x <= 1/e, so the subtraction loses < 1 bit); rho as a product with the hardware
// reciprocal; one hardware log2.  Each rho carries a relative error below ~8 ulp, so
// the site term is off by < 1.5e-6 in absolute value (the lattice sum stays FP64).
__device__ __forceinline__ float expm1_neg_f(float x) {
    return x > -1.0f ? expm1_taylor(x) : __builtin_amdgcn_exp2f(1.44269504088896341f * x) - 1.0f;
}

__device__ __forceinline__ float dec_rho_f(float s, float b1, float b2, float r0) {
    if (!(s > 0.0f)) return r0;
    return expm1_neg_f(-2.0f * b2 * s) * __builtin_amdgcn_rcpf(expm1_neg_f(-2.0f * b1 * s));
}

__device__ __forceinline__ float dec_log_ratio_f(float a, float c, float b1, float b2, float r0) {
    const float q = dec_rho_f(a, b1, b2, r0) * __builtin_amdgcn_rcpf(dec_rho_f(c, b1, b2, r0));
    return 0.693147180559945309f * __builtin_amdgcn_logf(q);
}

// Local field of site h (sublattice p) from the other sublattice, in the order
// +x, -x, +y, -y, +z, -z; the bond to -mu is stored at the neighbour.
template <typename T>
__device__ __forceinline__ void field(const T* __restrict__ s, const T* __restrict__ J, int NH,
                                      int h, int p, const Nbr& nb, T& Sx, T& Sy, T& Sz) {
    const T* o0 = s + (0 * 2 + (1 - p)) * NH;
    const T* o1 = s + (1 * 2 + (1 - p)) * NH;
    const T* o2 = s + (2 * 2 + (1 - p)) * NH;
    Sx = T(0);
    Sy = T(0);
    Sz = T(0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int mu = d >> 1;
        const T jj = (d & 1) ? J[(mu * 2 + (1 - p)) * NH + nb.n[d]] : J[(mu * 2 + p) * NH + h];
        const int idx = nb.n[d];
        Sx = fma(jj, o0[idx], Sx);
        Sy = fma(jj, o1[idx], Sy);
        Sz = fma(jj, o2[idx], Sz);
    }
}

template <typename T>
__device__ __forceinline__ double norm3(T x, T y, T z) {
    const double a = x, b = y, c = z;
    return sqrt(fma(c, c, fma(b, b, a * a)));
}

// Heat-bath of site h of configuration s (sublattice p) at beta with the given
// uniforms; returns s_new . S for the energy.
template <typename T>
__device__ __forceinline__ double reinsert_site(T* __restrict__ s, const T* __restrict__ J, int NH,
                                               int h, int p, const Nbr& nb, T beta, T r1, T r2) {
    T Sx, Sy, Sz, ox, oy, oz;
    field<T>(s, J, NH, h, p, nb, Sx, Sy, Sz);
    heatbath<T>(Sx, Sy, Sz, beta, r1, r2, ox, oy, oz);
    T* w0 = s + (0 * 2 + p) * NH;
    T* w1 = s + (1 * 2 + p) * NH;
    T* w2 = s + (2 * 2 + p) * NH;
    w0[h] = ox;
    w1[h] = oy;
    w2[h] = oz;
    const double dx = ox, dy = oy, dz = oz;
    return fma(dz, static_cast<double>(Sz), fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
}

// NT threads: 256 for one pair per workgroup (even / odd pairs), more for one chain
// per workgroup (ascending pairs, each waiting for the last one).
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_decimate(hsg_ensemble e, int pairing) {
    __shared__ double red[NT / 64];
    __shared__ int s_acc;
    const int L = e.L, N = L * L * L, NH = N / 2, NQ = N / 4;
    const int R = e.n_temps, C = e.n_chains;
    int ch, i_begin, i_end, i_step;
    if (pairing == 0) {
        ch = blockIdx.x;
        i_begin = 0;
        i_end = R - 1;
        i_step = 1;
    } else {
        const int first = pairing == 1 ? 0 : 1;
        const int n_sel = (R - 1 - first + 1) / 2;
        ch = blockIdx.x / n_sel;
        i_begin = first + 2 * (blockIdx.x % n_sel);
        i_end = i_begin + 1;
        i_step = 1;
    }
    const int smp = ch / C;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int d0 = static_cast<int>(philox(0u, n, cg, kTagDecimateRole << 24, k0, k1).w0 & 1u);

    for (int i = i_begin; i < i_end; i += i_step) {
        const int d = (d0 + i) & 1;
        const int x = label(sot[i], R, e.guard), y = label(sot[i + 1], R, e.guard);
        const size_t gx = static_cast<size_t>(ch) * R + x, gy = static_cast<size_t>(ch) * R + y;
        T* sx = static_cast<T*>(e.spins) + gx * 3 * N;
        T* sy = static_cast<T*>(e.spins) + gy * 3 * N;
        const double b1 = e.betas[i], b2 = e.betas[i + 1];
        const float fb1 = static_cast<float>(b1), fb2 = static_cast<float>(b2);
        const float fr0 = static_cast<float>(b2 / b1);

        double acc = 0.0;
        for (int h = threadIdx.x; h < NH; h += NT) {
            const Nbr nb = neighbours<0>(h, d, L);
            T ax, ay, az, cx, cy, cz;
            field<T>(sx, J, NH, h, d, nb, ax, ay, az);
            field<T>(sy, J, NH, h, d, nb, cx, cy, cz);
            const double a = norm3<T>(ax, ay, az), c = norm3<T>(cx, cy, cz);
            if constexpr (sizeof(T) == 4)  // the rearranged site term of the resident kernel
                acc += fma(b2 - b1, a - c,
                           static_cast<double>(dec_log_ratio_f(static_cast<float>(a), static_cast<float>(c), fb1, fb2, fr0)));
            else
                acc += (log_sinhc(b2 * a) - log_sinhc(b1 * a)) + (log_sinhc(b1 * c) - log_sinhc(b2 * c));
        }
        const double lnA = block_sum<NT>(acc, red);
        if (threadIdx.x == 0) {
            if (e.work) {
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2] = lnA;
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2 + 1] = static_cast<double>(d);
            }
            if (!isfinite(lnA)) atomicOr(e.guard, 1);
            const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, k0, k1);
            const bool ok = log(u01_52(w.w0, w.w1)) < lnA;
            st[2 * i] += 1;
            if (ok) {
                sot[i] = y;
                sot[i + 1] = x;
                tos[x] = i + 1;
                tos[y] = i;
                st[2 * i + 1] += 1;
            }
            s_acc = ok ? 1 : 0;
        }
        __syncthreads();
        if (s_acc) {
            // x goes to beta_2, y to beta_1; the kept sublattice is unchanged
            const uint32_t c3 = (kTagDecimate << 24) | (static_cast<uint32_t>(i) & 0xFFFFu);
            const T tb2 = static_cast<T>(b2), tb1 = static_cast<T>(b1);
            double ex = 0.0, ey = 0.0;
            if (sizeof(T) == 4) {
                for (int q = threadIdx.x; q < NQ; q += NT) {
                    const Words wx = philox(static_cast<uint32_t>(q), n, e.slot_base + static_cast<uint32_t>(gx), c3, k0, k1);
                    const Words wy = philox(static_cast<uint32_t>(q), n, e.slot_base + static_cast<uint32_t>(gy), c3, k0, k1);
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const int h = q + half * NQ;
                        const Nbr nb = neighbours<0>(h, d, L);
                        ex += reinsert_site<T>(sx, J, NH, h, d, nb, tb2,
                                               static_cast<T>(u01_23(half ? wx.w2 : wx.w0)),
                                               static_cast<T>(u01_23(half ? wx.w3 : wx.w1)));
                        ey += reinsert_site<T>(sy, J, NH, h, d, nb, tb1,
                                               static_cast<T>(u01_23(half ? wy.w2 : wy.w0)),
                                               static_cast<T>(u01_23(half ? wy.w3 : wy.w1)));
                    }
                }
            } else {
                for (int h = threadIdx.x; h < NH; h += NT) {
                    const Nbr nb = neighbours<0>(h, d, L);
                    const Words wx = philox(static_cast<uint32_t>(h), n, e.slot_base + static_cast<uint32_t>(gx), c3, k0, k1);
                    const Words wy = philox(static_cast<uint32_t>(h), n, e.slot_base + static_cast<uint32_t>(gy), c3, k0, k1);
                    ex += reinsert_site<T>(sx, J, NH, h, d, nb, tb2, static_cast<T>(u01_52(wx.w0, wx.w1)),
                                           static_cast<T>(u01_52(wx.w2, wx.w3)));
                    ey += reinsert_site<T>(sy, J, NH, h, d, nb, tb1, static_cast<T>(u01_52(wy.w0, wy.w1)),
                                           static_cast<T>(u01_52(wy.w2, wy.w3)));
                }
            }
            const double Hx = -block_sum<NT>(ex, red);
            const double Hy = -block_sum<NT>(ey, red);
            if (threadIdx.x == 0) {
                e.energy[gx] = Hx;
                e.energy[gy] = Hy;
                if (!isfinite(Hx) || !isfinite(Hy)) atomicOr(e.guard, 1);
            }
        }
        __syncthreads();  // spins, labels and energies of this pair are visible to the next
    }
}

// ---------------------------------------------------------------- LDS-resident variant
// Per pair, the kept sublattice of both configurations is staged into LDS with
// 16-byte loads ([config][mu][NH]); neighbour offsets use the compile-time L and
// every coupling is read once for both configurations.  Per site,
//   h(b2 s) - h(b1 s) = (b2 - b1) s + ln[expm1(-2 b2 s) / expm1(-2 b1 s)] - ln(b2/b1),
// and the ln(b2/b1) terms cancel between x and y, so the site contributes
//   (b2 - b1)(a - c) + ln[rho(a) / rho(c)],  rho(s) = expm1(-2 b2 s) / expm1(-2 b1 s),
// with one logarithm; rho -> b2/b1 as s -> 0 (its value at s = 0).
__device__ __forceinline__ double dec_rho(double s, double b1, double b2) {
    if (!(s > 0.0)) return b2 / b1;
    return expm1(-2.0 * b2 * s) / expm1(-2.0 * b1 * s);
}

// NT threads: 256 for one pair per workgroup (even / odd pairs, many workgroups),
// 1024 for one binary32 chain per workgroup (ascending pairs, each waiting for the
// last one).
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT, sizeof(T) == 4 && NT <= 256 ? 3 : 1) k_decimate_res(hsg_ensemble e, int pairing) {
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
    constexpr int NVP = NH * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per plane
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* kept = reinterpret_cast<T*>(smem_raw);  // [2][3][NH]
    __shared__ double red[NT / 64];
    __shared__ int s_acc;
    const int R = e.n_temps, C = e.n_chains;
    int ch, i_begin, i_end;
    if (pairing == 0) {
        ch = blockIdx.x;
        i_begin = 0;
        i_end = R - 1;
    } else {
        const int first = pairing == 1 ? 0 : 1;
        const int n_sel = (R - first) / 2;
        ch = blockIdx.x / n_sel;
        i_begin = first + 2 * (blockIdx.x % n_sel);
        i_end = i_begin + 1;
    }
    const int smp = ch / C;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(smp) * 3 * N;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int d0 = static_cast<int>(philox(0u, n, cg, kTagDecimateRole << 24, k0, k1).w0 & 1u);

    for (int i = i_begin; i < i_end; ++i) {
        const int d = (d0 + i) & 1;
        const int x = label(sot[i], R, e.guard), y = label(sot[i + 1], R, e.guard);
        const size_t gx = static_cast<size_t>(ch) * R + x, gy = static_cast<size_t>(ch) * R + y;
        T* sx = static_cast<T*>(e.spins) + gx * 3 * N;
        T* sy = static_cast<T*>(e.spins) + gy * 3 * N;
        const double b1 = e.betas[i], b2 = e.betas[i + 1];
        const float fb1 = static_cast<float>(b1), fb2 = static_cast<float>(b2);
        const float fr0 = static_cast<float>(b2 / b1);
        {
            const uint4* srcx = reinterpret_cast<const uint4*>(sx);
            const uint4* srcy = reinterpret_cast<const uint4*>(sy);
            uint4* dst = reinterpret_cast<uint4*>(kept);
            for (int v = threadIdx.x; v < 3 * NVP; v += NT) {
                const int mu = v / NVP, r = v - mu * NVP;
                const int src = (2 * mu + 1 - d) * NVP + r;
                dst[v] = srcx[src];
                dst[3 * NVP + v] = srcy[src];
            }
        }
        __syncthreads();
        double lin = 0.0, lg = 0.0;
        for (int h = threadIdx.x; h < NH; h += NT) {
            const Nbr nb = neighbours<L>(h, d, L);
            T ax = T(0), ay = T(0), az = T(0), cx = T(0), cy = T(0), cz = T(0);
#pragma unroll
            for (int dd = 0; dd < 6; ++dd) {
                const int mu = dd >> 1;
                const T jj = (dd & 1) ? J[(mu * 2 + (1 - d)) * NH + nb.n[dd]] : J[(mu * 2 + d) * NH + h];
                const int idx = nb.n[dd];
                ax = fma(jj, kept[0 * NH + idx], ax);
                ay = fma(jj, kept[1 * NH + idx], ay);
                az = fma(jj, kept[2 * NH + idx], az);
                cx = fma(jj, kept[3 * NH + idx], cx);
                cy = fma(jj, kept[4 * NH + idx], cy);
                cz = fma(jj, kept[5 * NH + idx], cz);
            }
            const double a = norm3<T>(ax, ay, az), c = norm3<T>(cx, cy, cz);
            lin += a - c;
            if constexpr (sizeof(T) == 4)
                lg += static_cast<double>(dec_log_ratio_f(static_cast<float>(a), static_cast<float>(c), fb1, fb2, fr0));
            else
                lg += log(dec_rho(a, b1, b2) / dec_rho(c, b1, b2));
        }
        const double lnA = block_sum<NT>(fma(b2 - b1, lin, lg), red);
        if (threadIdx.x == 0) {
            if (e.work) {
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2] = lnA;
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2 + 1] = static_cast<double>(d);
            }
            if (!isfinite(lnA)) atomicOr(e.guard, 1);
            const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, k0, k1);
            const bool ok = log(u01_52(w.w0, w.w1)) < lnA;
            st[2 * i] += 1;
            if (ok) {
                sot[i] = y;
                sot[i + 1] = x;
                tos[x] = i + 1;
                tos[y] = i;
                st[2 * i + 1] += 1;
            }
            s_acc = ok ? 1 : 0;
        }
        __syncthreads();
        if (s_acc) {
            const uint32_t c3 = (kTagDecimate << 24) | (static_cast<uint32_t>(i) & 0xFFFFu);
            const T tb[2] = {static_cast<T>(b2), static_cast<T>(b1)};  // x -> beta_2, y -> beta_1
            T* out[2] = {sx, sy};
            const uint32_t gs[2] = {e.slot_base + static_cast<uint32_t>(gx), e.slot_base + static_cast<uint32_t>(gy)};
            double en[2] = {0.0, 0.0};
            constexpr int NSITE = (sizeof(T) == 4) ? NQ : NH;  // one Philox block per site pair (binary32) or site
            for (int q = threadIdx.x; q < NSITE; q += NT) {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const Words w = philox(static_cast<uint32_t>(q), n, gs[r], c3, k0, k1);
#pragma unroll
                    for (int half = 0; half < (sizeof(T) == 4 ? 2 : 1); ++half) {
                        const int h = q + half * NQ;
                        const Nbr nb = neighbours<L>(h, d, L);
                        T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
                        for (int dd = 0; dd < 6; ++dd) {
                            const int mu = dd >> 1;
                            const T jj = (dd & 1) ? J[(mu * 2 + (1 - d)) * NH + nb.n[dd]] : J[(mu * 2 + d) * NH + h];
                            const int idx = nb.n[dd];
                            Sx = fma(jj, kept[(3 * r + 0) * NH + idx], Sx);
                            Sy = fma(jj, kept[(3 * r + 1) * NH + idx], Sy);
                            Sz = fma(jj, kept[(3 * r + 2) * NH + idx], Sz);
                        }
                        T r1, r2;
                        if (sizeof(T) == 4) {
                            r1 = static_cast<T>(u01_23(half ? w.w2 : w.w0));
                            r2 = static_cast<T>(u01_23(half ? w.w3 : w.w1));
                        } else {
                            r1 = static_cast<T>(u01_52(w.w0, w.w1));
                            r2 = static_cast<T>(u01_52(w.w2, w.w3));
                        }
                        T ox, oy, oz;
                        heatbath<T>(Sx, Sy, Sz, tb[r], r1, r2, ox, oy, oz);
                        out[r][(0 * 2 + d) * NH + h] = ox;
                        out[r][(1 * 2 + d) * NH + h] = oy;
                        out[r][(2 * 2 + d) * NH + h] = oz;
                        const double dx = ox, dy = oy, dz = oz;
                        en[r] += fma(dz, static_cast<double>(Sz),
                                     fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
                    }
                }
            }
            const double Hx = -block_sum<NT>(en[0], red);
            const double Hy = -block_sum<NT>(en[1], red);
            if (threadIdx.x == 0) {
                e.energy[gx] = Hx;
                e.energy[gy] = Hy;
                if (!isfinite(Hx) || !isfinite(Hy)) atomicOr(e.guard, 1);
            }
        }
        __syncthreads();  // the next pair restages the LDS and may read these spins
    }
}

// ---------------------------------------------------------------- staged ascending pass
// Binary32 ascending pass (one 1024-thread workgroup per chain) with every load of the
// pair loop taken off its critical path.  The chain's couplings sit in LDS for the
// whole pass (48 KB at L = 16), beside four buffers of one sublattice's three planes
// (24 KB each): the current pair's kept planes of its lower and upper configuration,
// and two staging buffers.  Pair i keeps sublattice 1 - d and pair i + 1 keeps d, so
// when pair i starts, the planes of sublattice d that pair i + 1 will keep are
// requested straight from HBM into LDS (loads that bypass the registers): those of the
// configuration at beta_{i+2} (pair i cannot touch it) into one staging buffer, those
// of the configuration at beta_{i+1} (pair i's upper one, the lower one of pair i + 1
// if pair i is rejected) into the other.  If pair i is accepted, its lower configuration
// moves to beta_{i+1} and its sublattice d is drawn anew: the new spins are written over
// that second buffer as well as to HBM, so either way the next pair's lower planes are
// in it.  The decision uniforms of all pairs, which do not depend on the states, are
// drawn up front.  Labels live in LDS too; barriers are LDS-only, so the staged loads
// stay in flight across them until the wait before the re-insertion.  Site
// arithmetic, its order and the reductions are k_decimate_res's, so results are the
// same bit for bit.
constexpr int kPfThreads = 1024;
constexpr int kPfMaxPairs = 256;

template <int L>
__global__ void __launch_bounds__(kPfThreads) k_decimate_pf(hsg_ensemble e) {
    using T = float;
    constexpr int NT = kPfThreads;
    constexpr int N = L * L * L, NH = N / 2, NQ = N / 4;
    constexpr int NVP = NH * static_cast<int>(sizeof(T)) / 16;  // 16-byte vectors per plane
    constexpr int NVB = 3 * NVP;                                 // per buffer
    static_assert(NVB % 64 == 0, "whole waves of staged vectors");
    static_assert(NQ <= NT && NH <= 2 * NT, "one re-insertion site pair and two terms per thread at most");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Js = reinterpret_cast<T*>(smem_raw);  // [3][2][NH]
    T* pool = Js + 3 * N;                    // [4][3][NH]
    __shared__ double red[2 * (NT / 64)];
    __shared__ double s_logu[kPfMaxPairs];
    __shared__ double s_beta[kPfMaxPairs + 1];
    __shared__ long long s_st[2 * kPfMaxPairs];
    __shared__ int s_sot[kPfMaxPairs + 1];
    __shared__ int s_acc;
    const int R = e.n_temps, C = e.n_chains;
    const int ch = blockIdx.x;
    const int t = static_cast<int>(threadIdx.x);
    const int wave_base = t & ~63;
    const int smp = ch / C;
    int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
    int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int d0 = static_cast<int>(philox(0u, n, cg, kTagDecimateRole << 24, k0, k1).w0 & 1u);
    const uint4* gsp = static_cast<const uint4*>(e.spins);

    for (int i = t; i < R - 1; i += NT) {
        const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, k0, k1);
        s_logu[i] = log(u01_52(w.w0, w.w1));
    }
    for (int i = t; i < R; i += NT) {
        s_sot[i] = label(sot[i], R, e.guard);
        s_beta[i] = e.betas[i];
    }
    for (int i = t; i < 2 * (R - 1); i += NT) s_st[i] = st[i];
    {
        const uint4* src = reinterpret_cast<const uint4*>(static_cast<const T*>(e.couplings) +
                                                          static_cast<size_t>(smp) * 3 * N);
        uint4* dst = reinterpret_cast<uint4*>(Js);
        for (int v = t; v < 6 * NVP; v += NT) dst[v] = src[v];
    }
    __syncthreads();
    auto buf = [&](int b) { return pool + static_cast<size_t>(b) * 3 * NH; };
    // planes of sublattice p of the chain's configuration in slot `slot` -> buffer b
    auto stage_now = [&](int b, int slot, int p) {
        const uint4* src = gsp + (static_cast<size_t>(ch) * R + slot) * 3 * N / 4;
        uint4* dst = reinterpret_cast<uint4*>(buf(b));
        for (int v = t; v < NVB; v += NT) {
            const int mu = v / NVP, r = v - mu * NVP;
            dst[v] = src[(2 * mu + p) * NVP + r];
        }
    };
    auto stage_ahead = [&](int b, int slot, int p) {
        const uint4* src = gsp + (static_cast<size_t>(ch) * R + slot) * 3 * N / 4;
        uint4* dst = reinterpret_cast<uint4*>(buf(b));
#pragma unroll
        for (int k = 0; k < (NVB + NT - 1) / NT; ++k) {
            const int v0 = k * NT + wave_base;  // this wave's first vector (64 consecutive)
            if (v0 < NVB) {
                const int v = v0 + (t & 63);
                const int mu = v / NVP, r = v - mu * NVP;
                __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + (2 * mu + p) * NVP + r),
                                                 (__attribute__((address_space(3))) void*)(dst + v0), 16, 0, 0);
            }
        }
    };
    int bl = 0, bu = 1, bp = 2, bn = 3;  // lower, upper, staging for the next lower / upper
    stage_now(bl, s_sot[0], 1 - (d0 & 1));
    stage_now(bu, s_sot[1], 1 - (d0 & 1));
    __syncthreads();

    for (int i = 0; i < R - 1; ++i) {
        const int d = (d0 + i) & 1;
        const int x = s_sot[i], y = s_sot[i + 1];
        const bool more = i + 2 < R;
        if (more) stage_ahead(bp, y, d);  // the other request goes out between the site terms
        const size_t gx = static_cast<size_t>(ch) * R + x, gy = static_cast<size_t>(ch) * R + y;
        T* sx = static_cast<T*>(e.spins) + gx * 3 * N;
        T* sy = static_cast<T*>(e.spins) + gy * 3 * N;
        const T* kx = buf(bl);
        const T* ky = buf(bu);
        const double b1 = s_beta[i], b2 = s_beta[i + 1];
        const float fb1 = static_cast<float>(b1), fb2 = static_cast<float>(b2);
        const float fr0 = static_cast<float>(b2 / b1);
        double lin = 0.0, lg = 0.0;
        auto term = [&](int h) {
            const Nbr nb = neighbours<L>(h, d, L);
            T ax = T(0), ay = T(0), az = T(0), cx = T(0), cy = T(0), cz = T(0);
#pragma unroll
            for (int dd = 0; dd < 6; ++dd) {
                const int mu = dd >> 1;
                const T jj = (dd & 1) ? Js[(mu * 2 + (1 - d)) * NH + nb.n[dd]] : Js[(mu * 2 + d) * NH + h];
                const int idx = nb.n[dd];
                ax = fma(jj, kx[0 * NH + idx], ax);
                ay = fma(jj, kx[1 * NH + idx], ay);
                az = fma(jj, kx[2 * NH + idx], az);
                cx = fma(jj, ky[0 * NH + idx], cx);
                cy = fma(jj, ky[1 * NH + idx], cy);
                cz = fma(jj, ky[2 * NH + idx], cz);
            }
            const double a = norm3<T>(ax, ay, az), c = norm3<T>(cx, cy, cz);
            lin += a - c;
            lg += static_cast<double>(dec_log_ratio_f(static_cast<float>(a), static_cast<float>(c), fb1, fb2, fr0));
        };
        // the memory pipeline is idle during the site terms: the second request goes
        // out between a thread's first and later sites (same summation order)
        if (t < NH) term(t);
        if (more) stage_ahead(bn, s_sot[i + 2], d);
        for (int h = t + NT; h < NH; h += NT) term(h);
        // ln A in block_sum's order; only thread 0 reads it, before the decision's barrier
        double lnA;
        {
            const double v = wave_sum(fma(b2 - b1, lin, lg));
            if ((t & 63) == 0) red[t >> 6] = v;
            lds_barrier();
            lnA = 0.0;
            if (t == 0)
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) lnA += red[w];
        }
        if (t == 0) {
            if (e.work) {
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2] = lnA;
                e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2 + 1] = static_cast<double>(d);
            }
            if (!isfinite(lnA)) atomicOr(e.guard, 1);
            const bool ok = s_logu[i] < lnA;
            st[2 * i] = s_st[2 * i] + 1;  // counts kept in LDS: no global read in the loop
            if (ok) {
                sot[i] = y;
                sot[i + 1] = x;
                s_sot[i] = y;
                s_sot[i + 1] = x;
                tos[x] = i + 1;
                tos[y] = i;
                st[2 * i + 1] = s_st[2 * i + 1] + 1;
            }
            s_acc = ok ? 1 : 0;
        }
        // this wave's staged planes have landed (requested at the start of the pair);
        // the barrier then makes every wave's visible, and the decision
        __builtin_amdgcn_s_waitcnt(0x0F70);  // gfx9 encoding: vmcnt = 0, expcnt = 7, lgkmcnt = 15
        lds_barrier();
        if (s_acc) {
            const uint32_t c3 = (kTagDecimate << 24) | (static_cast<uint32_t>(i) & 0xFFFFu);
            const T tb[2] = {static_cast<T>(b2), static_cast<T>(b1)};  // x -> beta_2, y -> beta_1
            const T* kin[2] = {kx, ky};
            T* out[2] = {sx, sy};
            T* nxt = buf(bp);  // x's new sublattice d: the next pair's lower planes
            const uint32_t gs[2] = {e.slot_base + static_cast<uint32_t>(gx), e.slot_base + static_cast<uint32_t>(gy)};
            double en[2] = {0.0, 0.0};
            for (int q = t; q < NQ; q += NT) {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const Words w = philox(static_cast<uint32_t>(q), n, gs[r], c3, k0, k1);
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const int h = q + half * NQ;
                        const Nbr nb = neighbours<L>(h, d, L);
                        T Sx = T(0), Sy = T(0), Sz = T(0);
#pragma unroll
                        for (int dd = 0; dd < 6; ++dd) {
                            const int mu = dd >> 1;
                            const T jj = (dd & 1) ? Js[(mu * 2 + (1 - d)) * NH + nb.n[dd]] : Js[(mu * 2 + d) * NH + h];
                            const int idx = nb.n[dd];
                            Sx = fma(jj, kin[r][0 * NH + idx], Sx);
                            Sy = fma(jj, kin[r][1 * NH + idx], Sy);
                            Sz = fma(jj, kin[r][2 * NH + idx], Sz);
                        }
                        const T r1 = static_cast<T>(u01_23(half ? w.w2 : w.w0));
                        const T r2 = static_cast<T>(u01_23(half ? w.w3 : w.w1));
                        T ox, oy, oz;
                        heatbath<T>(Sx, Sy, Sz, tb[r], r1, r2, ox, oy, oz);
                        out[r][(0 * 2 + d) * NH + h] = ox;
                        out[r][(1 * 2 + d) * NH + h] = oy;
                        out[r][(2 * 2 + d) * NH + h] = oz;
                        if (r == 0) {
                            nxt[0 * NH + h] = ox;
                            nxt[1 * NH + h] = oy;
                            nxt[2 * NH + h] = oz;
                        }
                        const double dx = ox, dy = oy, dz = oz;
                        en[r] += fma(dz, static_cast<double>(Sz),
                                     fma(dy, static_cast<double>(Sy), dx * static_cast<double>(Sx)));
                    }
                }
            }
            // both energies in one pass, each in block_sum's order (valid in thread 0)
            const double ex = wave_sum(en[0]), ey = wave_sum(en[1]);
            if ((t & 63) == 0) {
                red[t >> 6] = ex;
                red[NT / 64 + (t >> 6)] = ey;
            }
            lds_barrier();
            if (t == 0) {
                double sx = 0.0, sy = 0.0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) sx += red[w];
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) sy += red[NT / 64 + w];
                const double Hx = -sx, Hy = -sy;
                e.energy[gx] = Hx;
                e.energy[gy] = Hy;
                if (!isfinite(Hx) || !isfinite(Hy)) atomicOr(e.guard, 1);
            }
        }
        lds_barrier();  // the next pair reads the staged planes and reuses the others
        const int ol = bl, ou = bu;
        bl = bp;
        bu = bn;
        bp = ol;
        bn = ou;
    }
    // finish the call as k_decimate_finish does (every pair attempted: no diagnostics to
    // clear): the exchange counter, and each slot's round-trip state from its final
    // temperature, the inverse of the labels in LDS
    __shared__ int s_tos[kPfMaxPairs + 1];
    for (int r = t; r < R; r += NT) s_tos[r] = -1;
    lds_barrier();
    for (int i = t; i < R; i += NT) s_tos[s_sot[i]] = i;
    lds_barrier();
    if (t == 0) e.swap_ctr[ch] = n + 1u;
    for (int r = t; r < R; r += NT) {
        const int T = s_tos[r];
        const size_t k = static_cast<size_t>(ch) * R + r;
        int* rs = e.rt_state + k;
        long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + k;
        if (T == 0) {
            if (*rs == 2) *rtt += 1;
            *rs = 1;
        } else if (T == R - 1) {
            if (*rs == 1) *rs = 2;
        }
    }
}

// ---------------------------------------------------------------- split ascending pass
// With few chains, one workgroup per chain (k_decimate) leaves most CUs idle through
// the R - 1 sequential pairs.  Here pair i of every chain is spread over G workgroups,
// each owning a slice of the decimated sublattice, in two launches:
// k_dec_split_terms sums the site terms of each slice into a partial sum;
// k_dec_split_apply adds the G partial sums up in slice order (every workgroup of a
// chain alike, so all take the same decision), lets slice 0 record the decision, and
// on acceptance re-inserts its slice in both configurations, leaving per-slice energy
// sums that the next pair's first launch (or the finishing pass) adds up.  Per chain,
// in the scratch's partial area: G partial sums, 2 G energy sums, and a record of the
// pair's slots and decision.
struct DecSplit {
    double* part;  // [G]
    double* epart; // [G][2]
    int* rec;      // x, y, accepted
};

__device__ __forceinline__ DecSplit dec_split(const hsg_ensemble& e, int ch, int G) {
    const ScratchLayout sl = scratch_layout(e);
    double* base = reinterpret_cast<double*>(static_cast<unsigned char*>(e.scratch) + sl.partial) +
                   static_cast<size_t>(ch) * (3 * G + 2);
    DecSplit d;
    d.part = base;
    d.epart = base + G;
    d.rec = reinterpret_cast<int*>(base + 3 * G);
    return d;
}

// Energies of the configurations the previous pair re-inserted (if it was accepted).
__device__ __forceinline__ void dec_split_energies(const hsg_ensemble& e, int ch, int G, const DecSplit& d) {
    if (!d.rec[2]) return;
    double hx = 0.0, hy = 0.0;
    for (int g = 0; g < G; ++g) {
        hx += d.epart[2 * g];
        hy += d.epart[2 * g + 1];
    }
    const size_t base = static_cast<size_t>(ch) * e.n_temps;
    e.energy[base + d.rec[0]] = -hx;
    e.energy[base + d.rec[1]] = -hy;
    if (!isfinite(hx) || !isfinite(hy)) atomicOr(e.guard, 1);
}

template <typename T>
__global__ void __launch_bounds__(kDecThreads) k_dec_split_terms(hsg_ensemble e, int i, int G) {
    __shared__ double red[kDecThreads / 64];
    const int L = e.L, N = L * L * L, NH = N / 2;
    const int R = e.n_temps, C = e.n_chains;
    // a chain's slices on one XCD (they read each other's neighbouring sites)
    const int item = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int ch = item / G, g = item % G;
    const DecSplit ds = dec_split(e, ch, G);
    const int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int d = (static_cast<int>(philox(0u, n, cg, kTagDecimateRole << 24, k0, k1).w0 & 1u) + i) & 1;
    const int x = label(sot[i], R, e.guard), y = label(sot[i + 1], R, e.guard);
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(ch / C) * 3 * N;
    const T* sx = static_cast<const T*>(e.spins) + (static_cast<size_t>(ch) * R + x) * 3 * N;
    const T* sy = static_cast<const T*>(e.spins) + (static_cast<size_t>(ch) * R + y) * 3 * N;
    const double b1 = e.betas[i], b2 = e.betas[i + 1];
    const float fb1 = static_cast<float>(b1), fb2 = static_cast<float>(b2);
    const float fr0 = static_cast<float>(b2 / b1);
    const int h0 = static_cast<int>(static_cast<long long>(NH) * g / G);
    const int h1 = static_cast<int>(static_cast<long long>(NH) * (g + 1) / G);
    double acc = 0.0;
    for (int h = h0 + static_cast<int>(threadIdx.x); h < h1; h += kDecThreads) {
        const Nbr nb = neighbours<0>(h, d, L);
        T ax, ay, az, cx, cy, cz;
        field<T>(sx, J, NH, h, d, nb, ax, ay, az);
        field<T>(sy, J, NH, h, d, nb, cx, cy, cz);
        const double a = norm3<T>(ax, ay, az), c = norm3<T>(cx, cy, cz);
        if constexpr (sizeof(T) == 4)
            acc += fma(b2 - b1, a - c,
                       static_cast<double>(dec_log_ratio_f(static_cast<float>(a), static_cast<float>(c), fb1, fb2, fr0)));
        else
            acc += (log_sinhc(b2 * a) - log_sinhc(b1 * a)) + (log_sinhc(b1 * c) - log_sinhc(b2 * c));
    }
    const double part = block_sum<kDecThreads>(acc, red);
    if (threadIdx.x == 0) {
        ds.part[g] = part;
        if (g == 0) {
            if (i > 0) dec_split_energies(e, ch, G, ds);  // pair i - 1, before its record is replaced
            ds.rec[0] = x;
            ds.rec[1] = y;
            ds.rec[2] = 0;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kDecThreads) k_dec_split_apply(hsg_ensemble e, int i, int G) {
    __shared__ double red[kDecThreads / 64];
    const int L = e.L, N = L * L * L, NH = N / 2, NQ = N / 4;
    const int R = e.n_temps, C = e.n_chains;
    // a chain's slices on one XCD (they read each other's neighbouring sites)
    const int item = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int ch = item / G, g = item % G;
    const DecSplit ds = dec_split(e, ch, G);
    const uint32_t n = e.swap_ctr[ch];
    const uint32_t cg = e.chain_base + static_cast<uint32_t>(ch);
    const uint32_t k0 = key_lo(e.seed), k1 = key_hi(e.seed);
    const int d = (static_cast<int>(philox(0u, n, cg, kTagDecimateRole << 24, k0, k1).w0 & 1u) + i) & 1;
    const int x = ds.rec[0], y = ds.rec[1];
    double lnA = 0.0;
    for (int k = 0; k < G; ++k) lnA += ds.part[k];
    const Words w = philox(static_cast<uint32_t>(i), n, cg, kTagSwap << 24, k0, k1);
    const bool ok = log(u01_52(w.w0, w.w1)) < lnA;
    if (g == 0 && threadIdx.x == 0) {
        long long* st = reinterpret_cast<long long*>(e.swap_stats) + static_cast<size_t>(ch) * (R - 1) * 2;
        if (e.work) {
            e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2] = lnA;
            e.work[(static_cast<size_t>(ch) * (R - 1) + i) * 2 + 1] = static_cast<double>(d);
        }
        if (!isfinite(lnA)) atomicOr(e.guard, 1);
        st[2 * i] += 1;
        if (ok) {
            int* tos = e.temp_of_slot + static_cast<size_t>(ch) * R;
            int* sot = e.slot_of_temp + static_cast<size_t>(ch) * R;
            sot[i] = y;
            sot[i + 1] = x;
            tos[x] = i + 1;
            tos[y] = i;
            st[2 * i + 1] += 1;
            ds.rec[2] = 1;
        }
    }
    if (!ok) return;  // uniform over the chain's workgroups
    // x goes to beta_2, y to beta_1; this workgroup's slice of D is drawn anew
    const size_t gx = static_cast<size_t>(ch) * R + x, gy = static_cast<size_t>(ch) * R + y;
    T* sx = static_cast<T*>(e.spins) + gx * 3 * N;
    T* sy = static_cast<T*>(e.spins) + gy * 3 * N;
    const T* __restrict__ J = static_cast<const T*>(e.couplings) + static_cast<size_t>(ch / C) * 3 * N;
    const uint32_t c3 = (kTagDecimate << 24) | (static_cast<uint32_t>(i) & 0xFFFFu);
    const T tb2 = static_cast<T>(e.betas[i + 1]), tb1 = static_cast<T>(e.betas[i]);
    double ex = 0.0, ey = 0.0;
    if (sizeof(T) == 4) {  // one Philox block per site pair (q, q + N/4)
        const int q0 = static_cast<int>(static_cast<long long>(NQ) * g / G);
        const int q1 = static_cast<int>(static_cast<long long>(NQ) * (g + 1) / G);
        for (int q = q0 + static_cast<int>(threadIdx.x); q < q1; q += kDecThreads) {
            const Words wx = philox(static_cast<uint32_t>(q), n, e.slot_base + static_cast<uint32_t>(gx), c3, k0, k1);
            const Words wy = philox(static_cast<uint32_t>(q), n, e.slot_base + static_cast<uint32_t>(gy), c3, k0, k1);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int h = q + half * NQ;
                const Nbr nb = neighbours<0>(h, d, L);
                ex += reinsert_site<T>(sx, J, NH, h, d, nb, tb2, static_cast<T>(u01_23(half ? wx.w2 : wx.w0)),
                                       static_cast<T>(u01_23(half ? wx.w3 : wx.w1)));
                ey += reinsert_site<T>(sy, J, NH, h, d, nb, tb1, static_cast<T>(u01_23(half ? wy.w2 : wy.w0)),
                                       static_cast<T>(u01_23(half ? wy.w3 : wy.w1)));
            }
        }
    } else {
        const int h0 = static_cast<int>(static_cast<long long>(NH) * g / G);
        const int h1 = static_cast<int>(static_cast<long long>(NH) * (g + 1) / G);
        for (int h = h0 + static_cast<int>(threadIdx.x); h < h1; h += kDecThreads) {
            const Nbr nb = neighbours<0>(h, d, L);
            const Words wx = philox(static_cast<uint32_t>(h), n, e.slot_base + static_cast<uint32_t>(gx), c3, k0, k1);
            const Words wy = philox(static_cast<uint32_t>(h), n, e.slot_base + static_cast<uint32_t>(gy), c3, k0, k1);
            ex += reinsert_site<T>(sx, J, NH, h, d, nb, tb2, static_cast<T>(u01_52(wx.w0, wx.w1)),
                                   static_cast<T>(u01_52(wx.w2, wx.w3)));
            ey += reinsert_site<T>(sy, J, NH, h, d, nb, tb1, static_cast<T>(u01_52(wy.w0, wy.w1)),
                                   static_cast<T>(u01_52(wy.w2, wy.w3)));
        }
    }
    const double Ex = block_sum<kDecThreads>(ex, red);
    const double Ey = block_sum<kDecThreads>(ey, red);
    if (threadIdx.x == 0) {
        ds.epart[2 * g] = Ex;
        ds.epart[2 * g + 1] = Ey;
    }
}

// After every pair: advance the exchange counter, update round trips and clear the
// diagnostics of the pairs not attempted.  One thread per (chain, slot): thread r of
// a chain updates slot r's round-trip state from its final temperature, clears pair r
// if the pairing left it out, and (r = 0) advances the chain's counter.
// split_G > 0: the pass ran split over split_G workgroups per chain; the last pair's
// energies are added up here (thread r = 0).
__global__ void k_decimate_finish(hsg_ensemble e, int pairing, int split_G) {
    const int n_chains = e.n_samples * e.n_chains;
    const int R = e.n_temps;
    const long long b = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= static_cast<long long>(n_chains) * R) return;
    const int ch = static_cast<int>(b / R), r = static_cast<int>(b % R);
    if (r == 0) {
        if (split_G > 0) dec_split_energies(e, ch, split_G, dec_split(e, ch, split_G));
        e.swap_ctr[ch] += 1u;
    }
    if (e.work && r < R - 1) {
        const bool sel = pairing == 0 || (pairing == 1 ? (r % 2) == 0 : (r % 2) == 1);
        if (!sel) {
            e.work[(static_cast<size_t>(ch) * (R - 1) + r) * 2] = 0.0;
            e.work[(static_cast<size_t>(ch) * (R - 1) + r) * 2 + 1] = -1.0;
        }
    }
    const size_t k = static_cast<size_t>(ch) * R + r;
    const int T = e.temp_of_slot[k];
    int* rs = e.rt_state + k;
    long long* rtt = reinterpret_cast<long long*>(e.rt_trips) + k;
    if (T == 0) {
        if (*rs == 2) *rtt += 1;
        *rs = 1;
    } else if (T == R - 1) {
        if (*rs == 1) *rs = 2;
    }
}

template <typename T, int L, int NT>
static hipError_t go_decimate_nt(const hsg_ensemble& e, int pairing, int blocks, hipStream_t st) {
    constexpr size_t lds = 2 * 3 * (L * L * L / 2) * sizeof(T);
    auto kern = k_decimate_res<T, L, NT>;
    const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
    if (a != hipSuccess) return a;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, e, pairing);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t go_decimate_res(const hsg_ensemble& e, int pairing, int blocks, hipStream_t st, bool* finished) {
    if constexpr (std::is_same<T, float>::value && (L == 8 || L == 16)) {
        constexpr size_t lds = (3 * L * L * L + 4 * 3 * (L * L * L / 2)) * sizeof(float);
        if (pairing == 0 && e.n_temps - 1 <= kPfMaxPairs && lds <= max_block_lds()) {
            auto kern = k_decimate_pf<L>;
            const hipError_t a = allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds);
            if (a != hipSuccess) return a;
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(kPfThreads), lds, st, e);
            *finished = true;
            return hipGetLastError();
        }
    }
    // binary64 site terms need more than the 128 registers of a 1024-thread workgroup
    if (pairing == 0 && sizeof(T) == 4) return go_decimate_nt<T, L, 1024>(e, pairing, blocks, st);
    return go_decimate_nt<T, L, kDecThreads>(e, pairing, blocks, st);
}

// LDS-resident variant for L <= 16 (its two kept sublattices fit one workgroup's
// LDS), the generic kernel otherwise.
template <typename T>
static hipError_t go_decimate(const hsg_ensemble& e, int pairing, int blocks, hipStream_t st, bool* finished) {
    switch (e.L) {
        case 4: return go_decimate_res<T, 4>(e, pairing, blocks, st, finished);
        case 6: return go_decimate_res<T, 6>(e, pairing, blocks, st, finished);
        case 8: return go_decimate_res<T, 8>(e, pairing, blocks, st, finished);
        case 10: return go_decimate_res<T, 10>(e, pairing, blocks, st, finished);
        case 12: return go_decimate_res<T, 12>(e, pairing, blocks, st, finished);
        case 14: return go_decimate_res<T, 14>(e, pairing, blocks, st, finished);
        case 16: return go_decimate_res<T, 16>(e, pairing, blocks, st, finished);
        default:
            if (pairing == 0)  // binary64 with 512 threads (register budget, as above)
                hipLaunchKernelGGL((k_decimate<T, sizeof(T) == 4 ? 1024 : 512>), dim3(blocks),
                                   dim3(sizeof(T) == 4 ? 1024 : 512), 0, st, e, pairing);
            else
                hipLaunchKernelGGL((k_decimate<T, kDecThreads>), dim3(blocks), dim3(kDecThreads), 0, st, e, pairing);
            return hipGetLastError();
    }
}

// Workgroups per chain for the split ascending pass (L > 16, scratch given): enough
// to give the whole launch about 512 workgroups, at least 512 sites of D per
// workgroup, within the scratch's partial area; 1 = use k_decimate.
static int split_groups(const hsg_ensemble& e) {
    if (e.L <= 16 || e.scratch == nullptr) return 1;
    const int chains = e.n_samples * e.n_chains;
    const long long NH = static_cast<long long>(e.L) * e.L * e.L / 2;
    const ScratchLayout sl = scratch_layout(e);
    const long long per_chain = static_cast<long long>(e.n_temps) * sl.max_tiles;  // doubles
    long long G = (512 + chains - 1) / chains;
    G = G < NH / 512 ? G : NH / 512;
    G = G < (per_chain - 2) / 3 ? G : (per_chain - 2) / 3;
    return G < 2 ? 1 : static_cast<int>(G);
}

static unsigned finish_blocks(const hsg_ensemble& e) {
    const long long n = static_cast<long long>(e.n_samples) * e.n_chains * e.n_temps;
    return static_cast<unsigned>((n + 255) / 256);
}

hipError_t launch_decimate(const hsg_ensemble& e, int pairing, hipStream_t st) {
    const int chains = e.n_samples * e.n_chains;
    const int R = e.n_temps;
    if (chains <= 0 || R < 2) return hipSuccess;
    const int G = pairing == 0 ? split_groups(e) : 1;
    if (G > 1) {
        for (int i = 0; i < R - 1; ++i) {
            if (e.precision == HSG_FP64) {
                hipLaunchKernelGGL(k_dec_split_terms<double>, dim3(chains * G), dim3(kDecThreads), 0, st, e, i, G);
                hipLaunchKernelGGL(k_dec_split_apply<double>, dim3(chains * G), dim3(kDecThreads), 0, st, e, i, G);
            } else {
                hipLaunchKernelGGL(k_dec_split_terms<float>, dim3(chains * G), dim3(kDecThreads), 0, st, e, i, G);
                hipLaunchKernelGGL(k_dec_split_apply<float>, dim3(chains * G), dim3(kDecThreads), 0, st, e, i, G);
            }
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
        hipLaunchKernelGGL(k_decimate_finish, dim3(finish_blocks(e)), dim3(256), 0, st, e, pairing, G);
        return hipGetLastError();
    }
    int blocks = chains;
    if (pairing != 0) {
        const int first = pairing == 1 ? 0 : 1;
        const int n_sel = (R - 1 - first + 1) / 2;
        blocks = chains * n_sel;
    }
    bool finished = false;  // the staged ascending kernel finishes the call itself
    if (blocks > 0) {
        hipError_t err = e.precision == HSG_FP64 ? go_decimate<double>(e, pairing, blocks, st, &finished)
                                                 : go_decimate<float>(e, pairing, blocks, st, &finished);
        if (err != hipSuccess) return err;
    }
    if (finished) return hipSuccess;
    hipLaunchKernelGGL(k_decimate_finish, dim3(finish_blocks(e)), dim3(256), 0, st, e, pairing, 0);
    return hipGetLastError();
}

}  // namespace hsg
