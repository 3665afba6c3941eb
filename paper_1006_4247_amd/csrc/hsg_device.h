// Device-side building blocks of the hsgpt library (gfx950, wave64).
//
//  * Philox4x32-10 counter-based generator (Salmon et al., SC'11)
//  * uniform maps (23-bit binary32, 52-bit binary64, both open intervals)
//  * sublattice index arithmetic of the W/B checkerboard (paper Sec. III.A)
//  * single-site heat-bath and overrelaxation updates (paper Sec. III.C)
//  * deterministic wave64 + LDS block reductions in FP64
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hsgpt.h"

namespace hsg {

constexpr uint32_t kTagCoupling = 1u;
constexpr uint32_t kTagInit = 2u;
constexpr uint32_t kTagHeatbath = 3u;
constexpr uint32_t kTagSwap = 4u;

// ---------------------------------------------------------------- Philox4x32-10
struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
        const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ float u01_23(uint32_t w) {
    return (static_cast<float>(w >> 9) + 0.5f) * 1.1920928955078125e-07f;  // 2^-23
}

__device__ __forceinline__ double u01_52(uint32_t hi, uint32_t lo) {
    const uint64_t m = (static_cast<uint64_t>(hi) << 20) | static_cast<uint64_t>(lo >> 12);
    return (static_cast<double>(m) + 0.5) * 2.220446049250313080847263336181640625e-16;  // 2^-52
}

__host__ __device__ __forceinline__ uint32_t key_lo(uint64_t seed) {
    return static_cast<uint32_t>(seed & 0xFFFFFFFFull);
}
__host__ __device__ __forceinline__ uint32_t key_hi(uint64_t seed) {
    return static_cast<uint32_t>(seed >> 32);
}

// ---------------------------------------------------------------- lattice
// Sublattice index h = floor(i/2) + (L/2)(j + L k).  Neighbours of (h, parity p)
// in the other sublattice, order +x, -x, +y, -y, +z, -z.
struct Nbr {
    int n[6];
};

template <int LT>
__device__ __forceinline__ Nbr neighbours(int h, int p, int Lrt) {
    const int L = LT > 0 ? LT : Lrt;
    const int HL = L / 2;
    const int ih = h % HL;
    const int row = h / HL;  // j + L k
    const int j = row % L;
    const int k = row / L;
    const int o = (p + j + k) & 1;  // i = 2 ih + o
    int ixp = ih + o;
    if (ixp == HL) ixp = 0;
    int ixm = ih - 1 + o;
    if (ixm < 0) ixm = HL - 1;
    const int jp = (j == L - 1) ? 0 : j + 1;
    const int jm = (j == 0) ? L - 1 : j - 1;
    const int kp = (k == L - 1) ? 0 : k + 1;
    const int km = (k == 0) ? L - 1 : k - 1;
    Nbr r;
    r.n[0] = row * HL + ixp;
    r.n[1] = row * HL + ixm;
    r.n[2] = (jp + L * k) * HL + ih;
    r.n[3] = (jm + L * k) * HL + ih;
    r.n[4] = (j + L * kp) * HL + ih;
    r.n[5] = (j + L * km) * HL + ih;
    return r;
}

// Workgroups are dispatched to the eight XCDs round-robin (workgroup b on XCD
// b mod 8), and each XCD has its own L2.  Renumbering b so that XCD x receives
// the contiguous work items [x n/8, (x + 1) n/8) keeps work items that share
// data (replicas of one sample read the same couplings) on one L2.  A
// bijection of [0, n); the identity when n is not a multiple of 8.
__device__ __forceinline__ int xcd_order(int b, int n) {
    if (n & 7) return b;
    return (b & 7) * (n >> 3) + (b >> 3);
}

// ---------------------------------------------------------------- math wrappers
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float d_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }  // x >= 2^-126
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
// sin and cos of 2 pi r for r in [0, 1): the binary32 form uses the hardware
// sine/cosine, whose argument is in turns (absolute error ~1.3e-7 over every
// 23-bit uniform).
__device__ __forceinline__ void d_sincos_turns(float r, float* s, float* c) {
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void d_sincos_turns(double r, double* s, double* c) {
    sincospi(2.0 * r, s, c);
}
// Reciprocal: hardware approximation (1 ulp) in binary32, exact in binary64.
__device__ __forceinline__ float d_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double d_rcp(double x) { return 1.0 / x; }

// ---------------------------------------------------------------- single-site updates
// Heat-bath (paper Sec. III.C).  With R = beta |S| the component c of the new
// spin along n = S/|S| has density ~ exp(R c) on [-1, 1]; inverting its
// distribution function gives 1 - c = -log1p((1 - r1) expm1(-2R)) / R, which
// equals the paper's ln(z + (1/z - z) r1)/R, z = exp(-R), without overflow or
// cancellation.  R == 0 (beta = 0 or S = 0): c uniform, 1 - c = 2 (1 - r1).
// The orthogonal part sqrt(1 - c^2) (sin phi e1 + cos phi e2), phi = 2 pi r2,
// uses the branch-free frame of Duff et al. (JCGT 2017), sign +1 iff n_z >= 0.
//
// The angles (c, sin theta) are evaluated so that they keep full relative
// precision in every regime; in binary32 the single expression above would lose
// the small r1 to the rounding of 1 - r1 when R is large (errors ~1e-8/(r1 R)).
// The sign of c is known before any logarithm: c < 0 iff r1 < 1/(1 + e^R) =
// t/(1 + t), t = e^-R.  The distance u from the nearer pole is then
//   c >= 0: u = 1 - c = -ln(1 + a)/R,  a = (1 - r1) expm1(-2R)  in (-1, 0]
//   c <  0: u = 1 + c =  ln(1 + a)/R,  a = r1 expm1(2R)         in [0, e^R)
// and sin theta = sqrt(u (2 - u)), free of cancellation at both poles.  Each
// lane evaluates one expm1 and one ln(1 + a).  The argument y = 1 + a is formed
// as 1 + a (c < 0) or as r1 + (1 - r1) e^-2R, a sum of positive terms (c >= 0);
// ln(1 + a) = ln(y) a/(y - 1), y - 1 exact for y in [1/2, 2], the hardware log2
// (within 1 ulp relative over [1/2, 2], also next to 1) corrected by a/(y - 1)
// for the rounding of y (Goldberg, "What every computer scientist should know
// about floating-point arithmetic", 1991), or a itself when y rounds to 1: one
// branch-free evaluation for every lane.  expm1(x) by its Taylor series to x^10
// for |x| < 1, else from t^2 or its reciprocal.
// The exponent rounding of t costs a relative error ~2R 2^-24 in e^-2R, which
// the division by R turns into an absolute error below 1e-7 in u.  Measured worst
// case over 8.4 M (R, r1) samples spanning every regime (R from 1e-8 to ~60, r1 at
// the sign change of c): |dc| < 5.2e-7, |d sin theta| < 2e-7 (relative < 3.3e-7).
__device__ __forceinline__ float expm1_taylor(float x) {  // |x| < 1
    float p = 2.755731922e-7f;          // 1/10!
    p = fmaf(p, x, 2.755731922e-6f);    // 1/9!
    p = fmaf(p, x, 2.480158730e-5f);    // 1/8!
    p = fmaf(p, x, 1.984126984e-4f);    // 1/7!
    p = fmaf(p, x, 1.388888889e-3f);    // 1/6!
    p = fmaf(p, x, 8.333333333e-3f);    // 1/5!
    p = fmaf(p, x, 4.166666667e-2f);    // 1/4!
    p = fmaf(p, x, 1.666666667e-1f);    // 1/3!
    p = fmaf(p, x, 0.5f);
    p = fmaf(p, x, 1.0f);
    return p * x;
}

__device__ __forceinline__ void heatbath_angles(float R, float r1, float& c, float& st) {
    const float om = 1.0f - r1;
    float u;
    bool neg;
    if (R >= 1e-30f) {
        const float t = __builtin_amdgcn_exp2f(-1.44269504088896341f * R);
        const float E = t * t;
        neg = fmaf(r1, t, r1) < t;
        const float x = neg ? 2.0f * R : -2.0f * R;
        const float em = (R < 0.5f) ? expm1_taylor(x)
                                    : (neg ? __builtin_amdgcn_rcpf(E) : E) - 1.0f;
        const float a = (neg ? r1 : om) * em;
        const float y = neg ? 1.0f + a : fmaf(om, E, r1);
        const float ym1 = y - 1.0f;
        const float lg = ym1 == 0.0f ? a
                                     : 0.693147180559945309f * __builtin_amdgcn_logf(y) *
                                           (a * __builtin_amdgcn_rcpf(ym1));
        u = fabsf(lg) * __builtin_amdgcn_rcpf(R);
    } else {
        neg = r1 < 0.5f;
        u = neg ? 2.0f * r1 : 2.0f * om;
    }
    c = neg ? u - 1.0f : 1.0f - u;
    st = __builtin_amdgcn_sqrtf(u * (2.0f - u));
}

// Binary64: the single expression above is accurate to ~1e-16/(r1 R), far inside
// every tolerance, and matches the reference evaluation.
__device__ __forceinline__ void heatbath_angles(double R, double r1, double& c, double& st) {
    double w;
    if (R >= 1e-300) {
        w = -log1p((1.0 - r1) * expm1(-2.0 * R)) / R;
    } else {
        w = 2.0 * (1.0 - r1);
    }
    c = 1.0 - w;
    st = sqrt(w * (2.0 - w));
}

template <typename T>
__device__ __forceinline__ void heatbath(T Sx, T Sy, T Sz, T beta, T r1, T r2, T& ox, T& oy,
                                         T& oz) {
    const T ss = fma(Sz, Sz, fma(Sy, Sy, Sx * Sx));
    T nx = T(0), ny = T(0), nz = T(1), nrm = T(0);
    // binary32: the hardware reciprocal square root; a field below 1e-18 in norm
    // counts as zero (the draw is then uniform to within 1e-17 at any beta <= 10)
    if (ss > (sizeof(T) == 4 ? T(1e-36) : T(0))) {
        const T inv = d_rsqrt(ss);
        nx = Sx * inv;
        ny = Sy * inv;
        nz = Sz * inv;
        nrm = ss * inv;
    }
    T c, st;
    heatbath_angles(beta * nrm, r1, c, st);
    const T sgn = nz >= T(0) ? T(1) : T(-1);
    const T a = -d_rcp(sgn + nz);
    const T b = nx * ny * a;
    const T e1x = fma(sgn * nx, nx * a, T(1)), e1y = sgn * b, e1z = -sgn * nx;
    const T e2x = b, e2y = fma(ny, ny * a, sgn), e2z = -ny;
    T sp, cp;
    d_sincos_turns(r2, &sp, &cp);
    ox = fma(c, nx, st * fma(sp, e1x, cp * e2x));
    oy = fma(c, ny, st * fma(sp, e1y, cp * e2y));
    oz = fma(c, nz, st * fma(sp, e1z, cp * e2z));
}

// Overrelaxation (paper Sec. III.C): reflection about S; identity if S = 0.
template <typename T>
__device__ __forceinline__ void overrelax(T sx, T sy, T sz, T Sx, T Sy, T Sz, T& ox, T& oy,
                                          T& oz) {
    const T ss = fma(Sz, Sz, fma(Sy, Sy, Sx * Sx));
    if (ss > T(0)) {
        const T f = T(2) * fma(sz, Sz, fma(sy, Sy, sx * Sx)) * d_rcp(ss);
        ox = fma(f, Sx, -sx);
        oy = fma(f, Sy, -sy);
        oz = fma(f, Sz, -sz);
    } else {
        ox = sx;
        oy = sy;
        oz = sz;
    }
}

// Binary32 spins leave the unit sphere slowly under reflections alone (each one rounds;
// a heat-bath update writes a fresh unit vector), so sweeps without a heat-bath lattice
// sweep renormalise every spin once per sweep, in their last overrelaxation lattice
// sweep: s <- s / |s| with the hardware reciprocal square root (1 ulp).  Binary64 keeps
// |s| to ~1e-15 per thousand reflections and is left as it is.
__device__ __forceinline__ void renormalize(float& x, float& y, float& z) {
    const float r = __builtin_amdgcn_rsqf(fmaf(z, z, fmaf(y, y, x * x)));
    x *= r;
    y *= r;
    z *= r;
}
__device__ __forceinline__ void renormalize(double&, double&, double&) {}

// The library launches its kernels with its own copy of an ensemble descriptor, whose
// reserved0 word carries internal flags: bit 0 turns the renormalisation above off
// (hsg_tuning.flags & HSG_TUNE_NO_RENORM).
constexpr int32_t kFlagNoRenorm = 1;
__host__ __device__ __forceinline__ bool renorm_on(const hsg_ensemble& e) { return !(e.reserved0 & kFlagNoRenorm); }

template <typename T>
struct NormTol;
template <>
struct NormTol<float> {
    static constexpr double value = 1e-4;
};
template <>
struct NormTol<double> {
    static constexpr double value = 1e-10;
};

// ---------------------------------------------------------------- barriers
// Workgroup barrier for LDS traffic only: waits until this wave's LDS accesses
// have completed (lgkmcnt = 0), then joins the barrier.  Unlike __syncthreads()
// it does not wait for outstanding global loads and stores, so a prefetch or a
// write-back can stay in flight across it.  The empty asm statements with a
// memory clobber stop the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // gfx9 encoding: vmcnt = 63, expcnt = 7, lgkmcnt = 0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------- reductions
// One lane's binary64 value, as a wave-uniform value.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFll), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// The binary64 value of another lane of the same row of 16, by a DPP lane pattern.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 64 lanes of a wave (all active), every lane ending with the same bits:
// the butterfly that adds lane l and lane l ^ m for m = 1, 2, 4, 8, 16, 32 in turn.
// After the steps m < k every aligned group of k lanes holds one value, so any pattern
// that pairs each group with its neighbour group adds the same two values: within a row
// of 16 lanes the pairs come from DPP moves (quad permutations [1,0,3,2] and [2,3,0,1],
// then the half-row and row mirrors); across rows from one lane of each row, added as
// (row 0 + row 1) + (row 2 + row 3).  No LDS round trip.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // l ^ 1
    v += dpp_f64<0x4E>(v);   // l ^ 2
    v += dpp_f64<0x141>(v);  // half-row mirror: quads 0 and 1 of each half-row
    v += dpp_f64<0x140>(v);  // row mirror: the two half-rows of each row
    const double r01 = readlane_f64(v, 0) + readlane_f64(v, 16);
    const double r23 = readlane_f64(v, 32) + readlane_f64(v, 48);
    return r01 + r23;
}

// Deterministic block sum: fixed butterfly inside each wave, then wave partials
// added in wave order by thread 0.  `red` holds >= NT/64 doubles of LDS.  The
// result is valid in thread 0 only.  Contains two barriers (LDS-only ones if
// LDS_ONLY, see lds_barrier).
template <int NT, bool LDS_ONLY = false>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < (NT + 63) / 64; ++w) s += red[w];
    }
    if constexpr (LDS_ONLY) lds_barrier(); else __syncthreads();
    return s;
}

// ---------------------------------------------------------------- ensemble helpers
// Labels read from device memory index arrays: an out-of-range value latches
// the guard (bit 4) and is clamped, so it can never address outside a chain.
__device__ __forceinline__ int label(int v, int R, int* guard) {
    if (v < 0 || v >= R) {
        atomicOr(guard, 4);
        v = v < 0 ? 0 : R - 1;
    }
    return v;
}

__device__ __forceinline__ uint32_t heatbath_c3(int hs) {
    return (kTagHeatbath << 24) | ((static_cast<uint32_t>(hs) & 0xFFu) << 16);
}

// Scratch layout (bytes, each region aligned to 256):
//   candidate spins [slots][3][2][N/2] T | candidate energy [slots] double |
//   accept flags [slots] int32 | partial sums [slots][max_tiles] double |
//   work accumulators [slots] double | counters (256 bytes)
struct ScratchLayout {
    size_t cand, cand_energy, flags, partial, wacc, ctr, total;
    int max_tiles;
};

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

__host__ __device__ inline ScratchLayout scratch_layout(const hsg_ensemble& e) {
    ScratchLayout s;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const size_t slots = static_cast<size_t>(e.n_samples) * e.n_chains * e.n_temps;
    const size_t tsz = e.precision == HSG_FP64 ? 8 : 4;
    s.max_tiles = static_cast<int>((N / 4 + 63) / 64);
    if (s.max_tiles < 1) s.max_tiles = 1;
    size_t off = 0;
    s.cand = off;
    off += align256(slots * 3 * N * tsz);
    s.cand_energy = off;
    off += align256(slots * 8);
    s.flags = off;
    off += align256(slots * 4);
    s.partial = off;
    off += align256(slots * static_cast<size_t>(s.max_tiles) * 8);
    s.wacc = off;
    off += align256(slots * 8);
    s.ctr = off;  // work and barrier counters of the persistent batch launch
    off += 256;
    s.total = off;
    return s;
}

}  // namespace hsg
