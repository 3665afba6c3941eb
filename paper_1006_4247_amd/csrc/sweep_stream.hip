// Streaming sweep kernels: one launch per half-sweep, for lattices whose
// replica does not fit in one workgroup's LDS (L = 24, 32, ...).
//
// Work item = (group of RB replicas of one sample, tile of NT site pairs (h, h + N/4)
// of the updated sublattice), tiles fastest, in a one-dimensional grid whose blocks
// take the work items XCD by XCD (xcd_order): a replica's tiles run on one XCD, so
// the neighbouring z-planes a tile reads from its neighbours' ranges come from that
// XCD's L2.  A thread loads its sites' couplings once and reuses them for the RB
// replicas; neighbour spins of the other sublattice come through L1/L2 (each is read
// by six sites).  The energy
// of the last half-sweep of a sweep is reduced per tile into scratch and
// summed over tiles in a fixed order by a finalize kernel (deterministic).
#include <map>
#include <mutex>

#include "hsg_device.h"
#include "hsg_launch.h"
#include "stream_body.h"

namespace hsg {

template <typename T, int LT, int NT, int RB>
__global__ void __launch_bounds__(NT) k_stream_half(hsg_ensemble e, StreamArgs a) {
    __shared__ double red[(NT + 63) / 64];
    const int item = xcd_order(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    stream_tile<T, LT, NT, RB>(e, a, item % a.n_tiles, item / a.n_tiles, red);
}

// Sum the per-tile energies of every slot in tile order.  Regular: energy[] and
// (on the last sweep of the call) sweep_ctr += n_sweeps.  Annealing: the
// candidate energy of each active leg.
__global__ void k_stream_finalize(hsg_ensemble e, const double* part, int n_tiles, int anneal, int parity,
                                  int step, int ctr_add) {
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int slot;
    if (!anneal) {
        const int n_slots = e.n_samples * e.n_chains * e.n_temps;
        if (b >= n_slots) return;
        slot = b;
    } else {
        const int n_legs = e.n_samples * e.n_chains * ((e.n_temps - parity) / 2) * 2;
        if (b >= n_legs) return;
        const LegInfo li = leg_of_block(e, b, parity);
        if (step >= li.K) return;
        slot = li.slot;
    }
    double H = 0.0;
    for (int t = 0; t < n_tiles; ++t) H += part[static_cast<size_t>(slot) * sl.max_tiles + t];
    if (!isfinite(H)) atomicOr(e.guard, 1);
    if (!anneal) {
        e.energy[slot] = H;
        e.sweep_ctr[slot] += static_cast<uint32_t>(ctr_add);
    } else {
        reinterpret_cast<double*>(scr + sl.cand_energy)[slot] = H;
    }
}

// Annealing bookkeeping, one thread per leg.
//  phase 0: copy nothing, W = 0, candidate energy = current energy
//  phase 1 (step k): W += (next - cur) * H(candidate) for legs with k <= K
//  phase 2: work[] = W, sweep_ctr += K
__global__ void k_stream_anneal_book(hsg_ensemble e, int parity, int phase, int step) {
    const int n_legs = e.n_samples * e.n_chains * ((e.n_temps - parity) / 2) * 2;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_legs) return;
    const LegInfo li = leg_of_block(e, b, parity);
    const ScratchLayout sl = scratch_layout(e);
    unsigned char* scr = static_cast<unsigned char*>(e.scratch);
    double* wacc = reinterpret_cast<double*>(scr + sl.wacc);
    double* cen = reinterpret_cast<double*>(scr + sl.cand_energy);
    if (phase == 0) {
        wacc[li.slot] = 0.0;
        cen[li.slot] = e.energy[li.slot];
        const int raw = e.anneal_K[li.ipair];
        if (raw < 0 || raw > e.anneal_K_max) atomicOr(e.guard, 2);
    } else if (phase == 1) {
        if (step > li.K) return;
        const double cur = li.leg == 0 ? proto(e, li.ipair, li.K, step) : proto(e, li.ipair, li.K, li.K + 1 - step);
        const double nxt = li.leg == 0 ? proto(e, li.ipair, li.K, step + 1) : proto(e, li.ipair, li.K, li.K - step);
        wacc[li.slot] += (nxt - cur) * cen[li.slot];
    } else {
        e.work[(static_cast<size_t>(li.ch) * (e.n_temps - 1) + li.ipair) * 2 + li.leg] = wacc[li.slot];
        e.sweep_ctr[li.slot] += static_cast<uint32_t>(li.K);
    }
}

// Copy each leg's configuration into the candidate buffer (legs with K > 0).
template <typename T>
__global__ void k_stream_anneal_copy(hsg_ensemble e, int parity) {
    const LegInfo li = leg_of_block(e, blockIdx.x, parity);
    if (li.K == 0) return;
    const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
    const ScratchLayout sl = scratch_layout(e);
    const uint4* src = reinterpret_cast<const uint4*>(static_cast<const T*>(e.spins) + li.slot * 3 * N);
    uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<T*>(static_cast<unsigned char*>(e.scratch) + sl.cand) + li.slot * 3 * N);
    const size_t nv = 3 * N * sizeof(T) / 16;
    for (size_t v = threadIdx.x; v < nv; v += blockDim.x) dst[v] = src[v];
}

// ---------------------------------------------------------------- allocation-free form
// Device-resident storage for the per-tile energy sums of the streaming sweeps, for
// callers that cannot allocate (hsg_sweep_static).  Each device holds its own copy
// until the process ends; its address on the current device comes from
// hipGetSymbolAddress (the name itself is only a host-side stand-in).  Every tile
// writes its sum before the finalising pass reads it, so nothing needs clearing.
static __device__ __align__(256) double scratch[kStaticPartialDoubles];

namespace {
std::mutex g_static_mu;
std::map<int, double*> g_static_ptr;  // device -> address of `scratch` there
}  // namespace

hipError_t static_partial(double** out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> lock(g_static_mu);
    auto it = g_static_ptr.find(dev);
    if (it != g_static_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return err;
    g_static_ptr[dev] = static_cast<double*>(p);
    *out = static_cast<double*>(p);
    return hipSuccess;
}

// ---------------------------------------------------------------- dispatch
template <typename T, int LT, int NT, int RB>
static hipError_t launch_half(const hsg_ensemble& e, const StreamArgs& a, int gy, hipStream_t st) {
    hipLaunchKernelGGL((k_stream_half<T, LT, NT, RB>), dim3(a.n_tiles * gy), dim3(NT), 0, st, e, a);
    return hipGetLastError();
}

template <typename T, int NT, int RB>
static hipError_t half_L(const hsg_ensemble& e, const StreamArgs& a, int gy, hipStream_t st) {
    switch (e.L) {
    case 24: return launch_half<T, 24, NT, RB>(e, a, gy, st);
    case 32: return launch_half<T, 32, NT, RB>(e, a, gy, st);
    default: return launch_half<T, 0, NT, RB>(e, a, gy, st);
    }
}

template <typename T>
static hipError_t half_any(const hsg_ensemble& e, const StreamArgs& a, int gy, int nt, int rb,
                           hipStream_t st) {
    if (nt == 256 && rb == 1) return half_L<T, 256, 1>(e, a, gy, st);
    if (nt == 256 && rb == 2) return half_L<T, 256, 2>(e, a, gy, st);
    if (nt == 256 && rb == 4) return half_L<T, 256, 4>(e, a, gy, st);
    if (nt == 128 && rb == 1) return half_L<T, 128, 1>(e, a, gy, st);
    if (nt == 128 && rb == 4) return half_L<T, 128, 4>(e, a, gy, st);
    if (nt == 512 && rb == 1) return half_L<T, 512, 1>(e, a, gy, st);
    if (nt == 64 && rb == 1) return half_L<T, 64, 1>(e, a, gy, st);
    return hipErrorInvalidValue;
}

static hipError_t half_prec(const hsg_ensemble& e, const StreamArgs& a, int gy, int nt, int rb,
                            hipStream_t st) {
    if (e.precision == HSG_FP64) return half_any<double>(e, a, gy, nt, rb, st);
    return half_any<float>(e, a, gy, nt, rb, st);
}

// The per-tile energy sums of regular sweeps in `partial` (slots x max_tiles doubles),
// or in the caller's scratch if it is null.
hipError_t launch_stream_sweeps(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or,
                                int block_threads, int replicas_per_block, double* partial,
                                hipStream_t st, bool defer_last, int* n_tiles_out) {
    const int nt = block_threads > 0 ? block_threads : 256;
    int rb = replicas_per_block > 0 ? replicas_per_block : 1;
    const int CR = e.n_chains * e.n_temps;
    if (CR % rb != 0) rb = 1;
    const int NQ = e.L * e.L * e.L / 4;
    StreamArgs a{};
    a.n_tiles = (NQ + nt - 1) / nt;
    if (n_tiles_out) *n_tiles_out = a.n_tiles;
    a.partial = partial ? partial
                        : reinterpret_cast<double*>(static_cast<unsigned char*>(e.scratch) + scratch_layout(e).partial);
    const int n_slots = e.n_samples * CR;
    const int gy = n_slots / rb;
    const int nhalf = 2 * (n_hb + n_or);
    for (int k = 0; k < n_sweeps; ++k) {
        for (int pos = 0; pos < nhalf; ++pos) {
            a.hb[0] = a.hb[1] = pos < 2 * n_hb;
            a.par[0] = a.par[1] = pos & 1;
            a.hs[0] = a.hs[1] = pos;
            a.rn[0] = a.rn[1] = renorm_on(e) && n_hb == 0 && pos >= nhalf - 2;
            a.step = k;
            a.want = (pos == nhalf - 1);
            hipError_t err = half_prec(e, a, gy, nt, rb, st);
            if (err != hipSuccess) return err;
        }
        const int last = (k == n_sweeps - 1);
        if (last && defer_last) break;
        hipLaunchKernelGGL(k_stream_finalize, dim3((n_slots + 255) / 256), dim3(256), 0, st, e,
                           a.partial, a.n_tiles, 0, 0, k, last ? n_sweeps : 0);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_stream_anneal(const hsg_ensemble& e, int parity, int n_hb, int n_or,
                                int block_threads, hipStream_t st) {
    const int nt = block_threads > 0 ? block_threads : 256;
    const int R = e.n_temps;
    const int n_legs = e.n_samples * e.n_chains * ((R - parity) / 2) * 2;
    if (n_legs == 0) return hipSuccess;
    const int NQ = e.L * e.L * e.L / 4;
    const int nhalf = 2 * (n_hb + n_or);
    const int lb = (n_legs + 255) / 256;
    hipLaunchKernelGGL(k_stream_anneal_book, dim3(lb), dim3(256), 0, st, e, parity, 0, 0);
    if (e.precision == HSG_FP64)
        hipLaunchKernelGGL(k_stream_anneal_copy<double>, dim3(n_legs), dim3(256), 0, st, e, parity);
    else
        hipLaunchKernelGGL(k_stream_anneal_copy<float>, dim3(n_legs), dim3(256), 0, st, e, parity);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int Kmax = e.anneal_K_max;
    StreamArgs a{};
    a.anneal = 1;
    a.parity = parity;
    a.n_tiles = (NQ + nt - 1) / nt;
    a.partial = reinterpret_cast<double*>(static_cast<unsigned char*>(e.scratch) + scratch_layout(e).partial);
    for (int k = 0; k <= Kmax; ++k) {
        hipLaunchKernelGGL(k_stream_anneal_book, dim3(lb), dim3(256), 0, st, e, parity, 1, k);
        if (k == Kmax) break;
        for (int s = 0; s < nhalf; ++s) {
            const int up = s, dn = nhalf - 1 - s;  // forward / adjoint positions
            a.hb[0] = up < 2 * n_hb;
            a.par[0] = up & 1;
            a.hs[0] = up;
            a.hb[1] = dn < 2 * n_hb;
            a.par[1] = dn & 1;
            a.hs[1] = dn;
            a.rn[0] = renorm_on(e) && n_hb == 0 && up >= nhalf - 2;
            a.rn[1] = renorm_on(e) && n_hb == 0 && dn >= nhalf - 2;
            a.step = k;
            a.want = (s == nhalf - 1);
            err = half_prec(e, a, n_legs, nt, 1, st);
            if (err != hipSuccess) return err;
        }
        hipLaunchKernelGGL(k_stream_finalize, dim3(lb), dim3(256), 0, st, e, a.partial, a.n_tiles, 1,
                           parity, k, 0);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_stream_anneal_book, dim3(lb), dim3(256), 0, st, e, parity, 2, 0);
    return hipGetLastError();
}

}  // namespace hsg
