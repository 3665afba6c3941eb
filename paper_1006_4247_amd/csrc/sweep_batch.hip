// One persistent launch over the sweeps of an uneven batch: several size classes
// (ensembles of different L, sample counts and ladders) in one kernel.
//
// The grid is sized to stay resident (workgroups per CU from the occupancy query times
// the CUs) and split in two partitions.  Workgroups [0, G_s) run the classes whose
// replica does not fit one workgroup's LDS, half-sweep by half-sweep: in phase p every
// such class's tiles of half-sweep p are spread over the partition, which then meets at
// a barrier of its own before phase p + 1 (the phase barrier replaces the launch
// boundary between the streaming kernels' half-sweeps); the per-tile energies of each
// sweep's last half-sweep are summed after it.  Workgroups [G_s, G) take the replicas
// of the LDS-resident classes from a work counter, largest lattices first, and sweep
// each in LDS as k_resident does (L = 12, 14, 16; smaller lattices join the tiled
// half-sweeps); they never wait for the other partition.  Spins are
// bit for bit those of the per-class kernels (same site arithmetic and random
// numbers); energies agree up to the order of their FP64 sums.
//
// Work items (the work list): resident (class, replica); streaming (class, replica,
// tile) per half-sweep.  A streaming workgroup takes items of one XCD's contiguous
// share (workgroup b runs on XCD b mod 8), so the tiles of a replica meet in one L2.
//
// The barrier counter and the work counter live in the first ensemble's scratch
// (zeroed by a small kernel before each launch, never by a memset, so that the launch
// can be captured into graphs).  Waits are bounded: a wait that runs out (it cannot
// while the grid stays resident and nothing else holds the CUs for seconds) sets guard
// bit 16 and continues, so the kernel always ends.
#include <algorithm>

#include "hsg_device.h"
#include "hsg_launch.h"
#include "resident_body.h"
#include "stream_body.h"

namespace hsg {

constexpr int kBatchMax = 8;
constexpr int kBatchNT = 512;
constexpr int kGuardBatchWait = 16;

struct BatchArgs {
    hsg_ensemble e[kBatchMax];
    int kind[kBatchMax];     // 0 LDS-resident, 1 streaming
    int first[kBatchMax];    // first item of the class (resident: replicas; streaming: tiles)
    int n_tiles[kBatchMax];  // streaming: tiles per replica
    int n_classes;
    int n_res, n_str;        // resident items; streaming items per half-sweep
    int n_str_slots;         // replicas of the streaming classes
    int g_str;               // workgroups of the streaming partition (a multiple of 8, or 0)
    int n_sweeps, n_hb, n_or;
    unsigned int* ctr;       // [0] resident work counter, [1] streaming barrier arrivals
    uint32_t wait_limit;
};

__global__ void k_batch_reset(unsigned int* ctr) {
    if (threadIdx.x < 2) ctr[threadIdx.x] = 0u;
}

// Arrive at and wait for barrier number `k` (1, 2, ...) of the streaming partition.
__device__ __forceinline__ void partition_barrier(const BatchArgs& a, unsigned int k, int* guard) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's spins and sums, visible to every XCD
        atomicAdd(&a.ctr[1], 1u);
        const unsigned int target = k * static_cast<unsigned int>(a.g_str);
        uint32_t n = 0;
        // after one wait has run out, no workgroup waits again (the launch then ends
        // within one more time-out instead of one per barrier)
        while (__hip_atomic_load(&a.ctr[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target &&
               !(__hip_atomic_load(guard, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kGuardBatchWait)) {
            __builtin_amdgcn_s_sleep(2);
            if (++n > a.wait_limit) {
                atomicOr(guard, kGuardBatchWait);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

template <typename T, int LT>
__device__ __forceinline__ void batch_tile(const hsg_ensemble& e, const StreamArgs& sa, int tile, int group,
                                           double* red) {
    stream_tile<T, LT, kBatchNT, 1>(e, sa, tile, group, red);
}

template <typename T>
__device__ __forceinline__ void batch_tile_any(const hsg_ensemble& e, const StreamArgs& sa, int tile, int group,
                                               double* red) {
    switch (e.L) {
    case 24: batch_tile<T, 24>(e, sa, tile, group, red); break;
    case 32: batch_tile<T, 32>(e, sa, tile, group, red); break;
    default: batch_tile<T, 0>(e, sa, tile, group, red); break;
    }
}

// LDS-resident sizes of the batch: those whose replica keeps 512 threads busy (smaller
// lattices take the tiled half-sweeps with the streaming classes)
template <typename T>
__device__ __forceinline__ void batch_resident_any(const hsg_ensemble& e, int slot, const BatchArgs& a,
                                                   unsigned char* smem, double* red, double& s_H) {
    switch (e.L) {
    case 12: resident_item<T, 12, kBatchNT, 0, 0>(e, slot, a.n_sweeps, a.n_hb, a.n_or, 0, 0, smem, red, s_H); break;
    case 14: resident_item<T, 14, kBatchNT, 0, 0>(e, slot, a.n_sweeps, a.n_hb, a.n_or, 0, 0, smem, red, s_H); break;
    case 16: resident_item<T, 16, kBatchNT, 0, 0>(e, slot, a.n_sweeps, a.n_hb, a.n_or, 0, 0, smem, red, s_H); break;
    default: break;
    }
}

// class of item `it` among the classes of one kind (items numbered class by class)
__device__ __forceinline__ int class_of(const BatchArgs& a, int kind, int it) {
    int c = -1;
    for (int k = 0; k < a.n_classes; ++k)
        if (a.kind[k] == kind && it >= a.first[k]) c = k;
    return c;
}

template <typename T>
__global__ void __launch_bounds__(kBatchNT, 4) k_batch(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kBatchNT / 64];
    __shared__ double s_H;
    __shared__ int s_item;
    int* guard = a.e[0].guard;
    const int b = static_cast<int>(blockIdx.x);

    if (b >= a.g_str) {
        // LDS-resident classes: one replica per work item, from the counter
        for (;;) {
            if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(&a.ctr[0], 1u));
            __syncthreads();
            const int it = s_item;
            __syncthreads();
            if (it >= a.n_res) break;
            const int c = class_of(a, 0, it);
            batch_resident_any<T>(a.e[c], it - a.first[c], a, smem_raw, red, s_H);
            __syncthreads();
        }
        return;
    }

    // streaming classes: phases (half-sweeps) separated by the partition's barrier
    const int xcd = b & 7, rank = b >> 3, per_xcd = a.g_str >> 3;
    const int lo = static_cast<int>((static_cast<long long>(a.n_str) * xcd) >> 3);
    const int hi = static_cast<int>((static_cast<long long>(a.n_str) * (xcd + 1)) >> 3);
    const int nhalf = 2 * (a.n_hb + a.n_or);
    unsigned int nbar = 0;
    for (int k = 0; k < a.n_sweeps; ++k) {
        for (int pos = 0; pos < nhalf; ++pos) {
            for (int it = lo + rank; it < hi; it += per_xcd) {
                const int c = class_of(a, 1, it);
                const hsg_ensemble& e = a.e[c];
                const int local = it - a.first[c];
                StreamArgs sa{};
                sa.hb[0] = pos < 2 * a.n_hb;
                sa.par[0] = pos & 1;
                sa.hs[0] = pos;
                sa.rn[0] = renorm_on(e) && a.n_hb == 0 && pos >= nhalf - 2;
                sa.step = k;
                sa.want = (pos == nhalf - 1);
                sa.n_tiles = a.n_tiles[c];
                sa.partial = reinterpret_cast<double*>(static_cast<unsigned char*>(e.scratch) + scratch_layout(e).partial);
                batch_tile_any<T>(e, sa, local % a.n_tiles[c], local / a.n_tiles[c], red);
            }
            partition_barrier(a, ++nbar, guard);
        }
        // the sweep's energies: per replica, its tile sums in tile order
        for (int r = b * kBatchNT + static_cast<int>(threadIdx.x); r < a.n_str_slots; r += a.g_str * kBatchNT) {
            int c = -1, off = 0, base = 0;
            for (int q = 0; q < a.n_classes; ++q) {
                if (a.kind[q] != 1) continue;
                const int n = a.e[q].n_samples * a.e[q].n_chains * a.e[q].n_temps;
                if (c < 0 && r < base + n) {
                    c = q;
                    off = r - base;
                }
                base += n;
            }
            const hsg_ensemble& e = a.e[c];
            const ScratchLayout sl = scratch_layout(e);
            const double* part = reinterpret_cast<const double*>(static_cast<const unsigned char*>(e.scratch) + sl.partial);
            double H = 0.0;
            for (int t = 0; t < a.n_tiles[c]; ++t) H += part[static_cast<size_t>(off) * sl.max_tiles + t];
            if (!isfinite(H)) atomicOr(e.guard, 1);
            e.energy[off] = H;
            if (k == a.n_sweeps - 1) e.sweep_ctr[off] += static_cast<uint32_t>(a.n_sweeps);
        }
        // the next sweep's last half-sweep overwrites the sums only after seven more
        // barriers; the counters change after the last sweep only
    }
}

// ---------------------------------------------------------------- host side
// Classes swept in LDS by the batch kernel (the others take its tiled half-sweeps).
static bool batch_resident(const hsg_ensemble& e) {
    return resident_supported(e) && (e.L == 12 || e.L == 14 || e.L == 16);
}

bool batch_supported(const hsg_ensemble* ens, int n_ens) {
    if (n_ens < 1 || n_ens > kBatchMax) return false;
    for (int i = 0; i < n_ens; ++i) {
        if (ens[i].precision != ens[0].precision || ens[i].L < 4) return false;
        if (!batch_resident(ens[i]) && !ens[i].scratch) return false;
    }
    return ens[0].scratch != nullptr;
}

bool batch_needs_scratch(const hsg_ensemble& e) { return !batch_resident(e); }

template <typename T>
static hipError_t batch_go(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or, int g_str_req,
                           hipStream_t st) {
    BatchArgs a{};
    a.n_classes = n_ens;
    a.n_sweeps = n_sweeps;
    a.n_hb = n_hb;
    a.n_or = n_or;
    size_t lds = 0;
    double res_work = 0.0, str_work = 0.0;
    // resident classes first, largest lattices first (their replicas take longest)
    int order[kBatchMax];
    for (int i = 0; i < n_ens; ++i) order[i] = i;
    for (int i = 0; i < n_ens; ++i)
        for (int j = i + 1; j < n_ens; ++j)
            if (ens[order[j]].L > ens[order[i]].L) {
                const int t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
    int n_res = 0, n_str = 0, n_str_slots = 0;
    for (int k = 0; k < n_ens; ++k) {
        const int i = order[k];
        const hsg_ensemble& e = ens[i];
        a.e[k] = e;
        const int slots = e.n_samples * e.n_chains * e.n_temps;
        const size_t N = static_cast<size_t>(e.L) * e.L * e.L;
        if (batch_resident(e)) {
            a.kind[k] = 0;
            a.first[k] = n_res;
            n_res += slots;
            lds = std::max(lds, 3 * N * sizeof(T));
            res_work += static_cast<double>(slots) * N;
        } else {
            a.kind[k] = 1;
            a.n_tiles[k] = static_cast<int>((N / 4 + kBatchNT - 1) / kBatchNT);
            a.first[k] = n_str;
            n_str += slots * a.n_tiles[k];
            n_str_slots += slots;
            str_work += static_cast<double>(slots) * N;
        }
    }
    a.n_res = n_res;
    a.n_str = n_str;
    a.n_str_slots = n_str_slots;
    a.ctr = reinterpret_cast<unsigned int*>(static_cast<unsigned char*>(ens[0].scratch) + scratch_layout(ens[0]).ctr);
    a.wait_limit = 1u << 23;  // ~0.5 s of 2-unit sleeps

    auto kern = k_batch<T>;
    int per_cu = 1;
    hipError_t err = blocks_per_cu_query(reinterpret_cast<const void*>(kern), kBatchNT, lds, &per_cu);
    if (err != hipSuccess) return err;
    const int grid = device_cus() * per_cu;
    // streaming partition: proportional to the streaming classes' share of the updates,
    // weighted by their lower rate (a streaming update costs ~3x a resident one)
    int g_str = 0;
    if (n_str > 0) {
        if (g_str_req > 0) {
            g_str = g_str_req;
        } else {
            const double w = 3.0 * str_work / (3.0 * str_work + res_work);
            g_str = static_cast<int>(w * grid);
        }
        g_str = (g_str / 8) * 8;
        if (g_str < 8) g_str = 8;
        if (n_res > 0 && g_str > grid - 8) g_str = ((grid - 8) / 8) * 8;
        if (g_str > grid) g_str = (grid / 8) * 8;
    }
    a.g_str = g_str;
    const int launch = n_res > 0 ? grid : g_str;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, a.ctr);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(launch), dim3(kBatchNT), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_sweeps(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or, int g_str,
                               hipStream_t st) {
    if (ens[0].precision == HSG_FP64) return batch_go<double>(ens, n_ens, n_sweeps, n_hb, n_or, g_str, st);
    return batch_go<float>(ens, n_ens, n_sweeps, n_hb, n_or, g_str, st);
}

}  // namespace hsg
