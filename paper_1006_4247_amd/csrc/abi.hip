// C ABI of the hsgpt library: argument validation (before any launch),
// thread-local error reporting and dispatch to the kernel launchers.
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hsg_device.h"
#include "hsg_launch.h"

namespace {

thread_local char g_err[512] = "";

hsg_status fail(hsg_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

hsg_status ok() {
    g_err[0] = '\0';
    return HSG_OK;
}

hsg_status device(hipError_t err, const char* what) {
    if (err == hipSuccess) return ok();
    return fail(HSG_ERR_DEVICE, "%s: %s", what, hipGetErrorString(err));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

enum Need : unsigned { kState = 1u, kAnneal = 2u, kMeasure = 4u, kScratch = 8u };

hsg_status check_shape(const hsg_ensemble& e, int idx) {
    if (e.L < 2 || e.L > 64 || (e.L & 1))
        return fail(HSG_ERR_INVALID, "ensemble %d: L = %d must be even and in [2, 64]", idx, e.L);
    if (e.n_samples < 1 || e.n_chains < 1 || e.n_temps < 2)
        return fail(HSG_ERR_INVALID, "ensemble %d: need n_samples >= 1, n_chains >= 1, n_temps >= 2 (got %d, %d, %d)",
                    idx, e.n_samples, e.n_chains, e.n_temps);
    if (e.precision != HSG_FP64 && e.precision != HSG_FP32)
        return fail(HSG_ERR_INVALID, "ensemble %d: unknown precision %d", idx, e.precision);
    const long long slots = static_cast<long long>(e.n_samples) * e.n_chains * e.n_temps;
    if (slots * e.L * e.L * e.L * 3 > (1LL << 40) || slots > (1LL << 30))
        return fail(HSG_ERR_INVALID, "ensemble %d: too many sites", idx);
    return HSG_OK;
}

hsg_status check_one(const hsg_ensemble& e, int idx, unsigned need) {
    hsg_status st = check_shape(e, idx);
    if (st != HSG_OK) return st;
    const void* must[] = {e.spins, e.couplings, e.betas, e.temp_of_slot, e.slot_of_temp, e.energy,
                          e.sweep_ctr, e.swap_ctr, e.swap_stats, e.rt_state, e.rt_trips, e.guard};
    const char* names[] = {"spins", "couplings", "betas", "temp_of_slot", "slot_of_temp", "energy",
                           "sweep_ctr", "swap_ctr", "swap_stats", "rt_state", "rt_trips", "guard"};
    for (int k = 0; k < 12; ++k)
        if (!must[k]) return fail(HSG_ERR_INVALID, "ensemble %d: %s is NULL", idx, names[k]);
    if (!aligned(e.spins, 16) || !aligned(e.couplings, 16))
        return fail(HSG_ERR_INVALID, "ensemble %d: spins and couplings must be 16-byte aligned", idx);
    if (!aligned(e.betas, 8) || !aligned(e.energy, 8) || !aligned(e.swap_stats, 8) || !aligned(e.rt_trips, 8))
        return fail(HSG_ERR_INVALID, "ensemble %d: double/int64 arrays must be 8-byte aligned", idx);
    if (need & kAnneal) {
        if (!e.anneal_K || !e.work)
            return fail(HSG_ERR_INVALID, "ensemble %d: annealed exchange needs anneal_K and work", idx);
        if (e.anneal_K_max < 0 || e.anneal_K_max > 4096)
            return fail(HSG_ERR_INVALID, "ensemble %d: anneal_K_max = %d outside [0, 4096]", idx, e.anneal_K_max);
        if (e.anneal_lambda && e.anneal_K_max == 0)
            return fail(HSG_ERR_INVALID, "ensemble %d: anneal_lambda given with anneal_K_max = 0", idx);
    }
    if ((need & (kAnneal | kScratch)) && (!e.scratch || !aligned(e.scratch, 256)))
        return fail(HSG_ERR_INVALID, "ensemble %d: scratch (hsg_scratch_bytes bytes, 256-byte aligned) is required", idx);
    if (need & kMeasure) {
        if (!e.e_temp) return fail(HSG_ERR_INVALID, "ensemble %d: e_temp is NULL", idx);
        if (e.n_chains >= 2 && (!e.Q || !e.chi))
            return fail(HSG_ERR_INVALID, "ensemble %d: Q and chi are required with n_chains >= 2", idx);
    }
    return HSG_OK;
}

hsg_status check_all(const hsg_ensemble* ens, int n_ens, unsigned need) {
    if (!ens || n_ens < 1) return fail(HSG_ERR_INVALID, "need at least one ensemble (ens=%p, n_ens=%d)",
                                       static_cast<const void*>(ens), n_ens);
    for (int i = 0; i < n_ens; ++i) {
        hsg_status s = check_one(ens[i], i, need);
        if (s != HSG_OK) return s;
    }
    return HSG_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// 1: LDS-resident, persistent double-buffered; 3: LDS-resident, one workgroup per
// replica; 2: streaming half-sweeps; 4: wavefront over z-planes; 6: LDS-resident,
// persistent single-buffer; 0: 3 if a replica fits in LDS, else 2 (measured faster
// than 4 at L = 20 .. 40).
int sweep_path(const hsg_ensemble& e, const hsg_tuning* t) {
    const int path = t ? t->path : 0;
    if (path != 0) return path;
    if (hsg::resident_supported(e)) return 3;
    return 2;
}

// Every path but the streaming one works without the scratch.
bool use_resident(const hsg_ensemble& e, const hsg_tuning* t) { return sweep_path(e, t) != 2; }

// The library's own copy of a descriptor for the sweep kernels, its internal flag
// word set from the tuning (renormalisation of sweeps without heat-bath on unless
// HSG_TUNE_NO_RENORM).
hsg_ensemble launch_copy(const hsg_ensemble& e, const hsg_tuning* t = nullptr) {
    hsg_ensemble c = e;
    c.reserved0 = (t && (t->flags & HSG_TUNE_NO_RENORM)) ? hsg::kFlagNoRenorm : 0;
    return c;
}

}  // namespace

namespace hsg {
void set_last_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg ? msg : ""); }
}  // namespace hsg

extern "C" {

int hsg_abi_version(void) { return HSG_ABI_VERSION; }

const char* hsg_last_error(void) { return g_err; }

size_t hsg_scratch_bytes(const hsg_ensemble* ens) {
    if (!ens || check_shape(*ens, 0) != HSG_OK) return 0;
    return hsg::scratch_layout(*ens).total;
}

hsg_status hsg_init_couplings(const hsg_ensemble* ens, int n_ens, void* stream) {
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_init_couplings(ens[i], as_stream(stream));
        if (err != hipSuccess) return device(err, "init_couplings");
    }
    return ok();
}

hsg_status hsg_init_spins(const hsg_ensemble* ens, int n_ens, int cold, void* stream) {
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_init_spins(ens[i], cold, as_stream(stream));
        if (err != hipSuccess) return device(err, "init_spins");
    }
    return ok();
}

hsg_status hsg_sweep_tuned(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                           const hsg_tuning* tuning, void* stream) {
    if (n_sweeps < 0 || n_hb < 0 || n_hb > 127 || n_or < 0 || n_hb + n_or < 1)
        return fail(HSG_ERR_INVALID, "need n_sweeps >= 0, 0 <= n_hb <= 127, n_or >= 0, n_hb + n_or >= 1 (got %d, %d, %d)",
                    n_sweeps, n_hb, n_or);
    if (tuning && (tuning->path < 0 || tuning->path > 6 || tuning->block_threads < 0 ||
                   tuning->replicas_per_block < 0 || (tuning->flags & ~HSG_TUNE_NO_RENORM) != 0))
        return fail(HSG_ERR_INVALID, "bad tuning values");
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    if (tuning && tuning->path == 5) {
        if (n_ens > 8) return fail(HSG_ERR_UNSUPPORTED, "the persistent batch launch takes at most 8 ensembles");
        hsg_ensemble copy[8];
        for (int i = 0; i < n_ens; ++i) copy[i] = launch_copy(ens[i], tuning);
        if (!hsg::batch_supported(copy, n_ens))
            return fail(HSG_ERR_UNSUPPORTED,
                        "the persistent batch launch needs one precision, L >= 4, and the scratch of the first "
                        "ensemble and of every ensemble it sweeps in tiles (L other than 12, 14, 16)");
        for (int i = 0; i < n_ens; ++i) {
            s = check_one(ens[i], i, i == 0 || hsg::batch_needs_scratch(ens[i]) ? kScratch : 0u);
            if (s != HSG_OK) return s;
        }
        if (n_sweeps == 0) return ok();
        return device(hsg::launch_batch_sweeps(copy, n_ens, n_sweeps, n_hb, n_or, tuning->block_threads,
                                               as_stream(stream)),
                      "persistent batch sweep");
    }
    for (int i = 0; i < n_ens; ++i) {
        if (tuning && tuning->path == 1 && !hsg::persistent_supported(ens[i]))
            return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: L = %d does not fit the persistent LDS-resident path", i, ens[i].L);
        if (tuning && tuning->path == 3 && !hsg::resident_supported(ens[i]))
            return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: L = %d does not fit the LDS-resident path", i, ens[i].L);
        if (tuning && tuning->path == 4 && !hsg::wave_supported(ens[i]))
            return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: L = %d does not fit the wavefront path", i, ens[i].L);
        if (tuning && tuning->path == 6 && !hsg::chain_supported(ens[i]))
            return fail(HSG_ERR_UNSUPPORTED,
                        "ensemble %d: the persistent single-buffer path takes binary32 at L = 16", i);
        if (!use_resident(ens[i], tuning)) {
            s = check_one(ens[i], i, kScratch);
            if (s != HSG_OK) return s;
        }
    }
    if (n_sweeps == 0) return ok();
    for (int i = 0; i < n_ens; ++i) {
        const int nt = tuning ? tuning->block_threads : 0;
        hipError_t err;
        const int path = sweep_path(ens[i], tuning);
        const hsg_ensemble e = launch_copy(ens[i], tuning);
        if (path == 1) {
            err = hsg::launch_resident(e, n_sweeps, n_hb, n_or, 2, 0, nt, as_stream(stream));
        } else if (path == 3) {
            err = hsg::launch_resident(e, n_sweeps, n_hb, n_or, 0, 0, nt, as_stream(stream));
        } else if (path == 6) {
            err = hsg::launch_resident(e, n_sweeps, n_hb, n_or, 3, 0, nt, as_stream(stream));
        } else if (path == 4) {
            if (nt != 0) return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: the wavefront path takes no block_threads", i);
            err = hsg::launch_wave_sweeps(e, n_sweeps, n_hb, n_or, as_stream(stream));
        } else {
            const int rb = tuning ? tuning->replicas_per_block : 0;
            err = hsg::launch_stream_sweeps(e, n_sweeps, n_hb, n_or, nt, rb, nullptr, as_stream(stream));
        }
        if (err == hipErrorInvalidValue)
            return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: no kernel instance for block_threads = %d", i, nt);
        if (err != hipSuccess) return device(err, "sweep");
    }
    return ok();
}

hsg_status hsg_sweep(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                     void* stream) {
    return hsg_sweep_tuned(ens, n_ens, n_sweeps, n_hb, n_or, nullptr, stream);
}

hsg_status hsg_sweep_static(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                            void* stream) {
    if (n_sweeps < 0 || n_hb < 0 || n_hb > 127 || n_or < 0 || n_hb + n_or < 1)
        return fail(HSG_ERR_INVALID, "need n_sweeps >= 0, 0 <= n_hb <= 127, n_or >= 0, n_hb + n_or >= 1 (got %d, %d, %d)",
                    n_sweeps, n_hb, n_or);
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    bool any_stream = false;
    for (int i = 0; i < n_ens; ++i) {
        if (use_resident(ens[i], nullptr)) continue;
        any_stream = true;
        const hsg::ScratchLayout sl = hsg::scratch_layout(ens[i]);
        const size_t need = static_cast<size_t>(ens[i].n_samples) * ens[i].n_chains * ens[i].n_temps * sl.max_tiles;
        if (need > hsg::kStaticPartialDoubles)
            return fail(HSG_ERR_INVALID,
                        "ensemble %d: its per-tile energy sums need %zu bytes, more than the %zu bytes of the "
                        "library's device array (use hsg_sweep with a caller-allocated scratch)",
                        i, need * sizeof(double), hsg::kStaticPartialDoubles * sizeof(double));
    }
    double* partial = nullptr;
    if (any_stream) {
        hipError_t err = hsg::static_partial(&partial);
        if (err != hipSuccess) return device(err, "sweep_static: device array address");
    }
    if (n_sweeps == 0) return ok();
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err;
        const hsg_ensemble e = launch_copy(ens[i]);
        if (use_resident(e, nullptr))
            err = hsg::launch_resident(e, n_sweeps, n_hb, n_or, 0, 0, 0, as_stream(stream));
        else
            err = hsg::launch_stream_sweeps(e, n_sweeps, n_hb, n_or, 0, 0, partial, as_stream(stream));
        if (err != hipSuccess) return device(err, "sweep_static");
    }
    return ok();
}

hsg_status hsg_energy(const hsg_ensemble* ens, int n_ens, double* H_out, void* stream) {
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    if (H_out && !aligned(H_out, 8)) return fail(HSG_ERR_INVALID, "H_out must be 8-byte aligned");
    size_t off = 0;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_energy(ens[i], H_out ? H_out + off : nullptr, as_stream(stream));
        if (err != hipSuccess) return device(err, "energy");
        off += static_cast<size_t>(ens[i].n_samples) * ens[i].n_chains * ens[i].n_temps;
    }
    return ok();
}

hsg_status hsg_swap(const hsg_ensemble* ens, int n_ens, int pairing, void* stream) {
    if (pairing < 0 || pairing > 2) return fail(HSG_ERR_INVALID, "pairing must be 0, 1 or 2 (got %d)", pairing);
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i)
        if (ens[i].n_temps > 256) return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: n_temps > 256", i);
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_swap(ens[i], pairing, as_stream(stream));
        if (err != hipSuccess) return device(err, "swap");
    }
    return ok();
}

hsg_status hsg_anneal_swap(const hsg_ensemble* ens, int n_ens, int parity, int n_hb, int n_or,
                           void* stream) {
    if (parity < 0 || parity > 1) return fail(HSG_ERR_INVALID, "parity must be 0 or 1 (got %d)", parity);
    if (n_hb < 0 || n_hb > 127 || n_or < 0 || n_hb + n_or < 1)
        return fail(HSG_ERR_INVALID, "need 0 <= n_hb <= 127, n_or >= 0, n_hb + n_or >= 1");
    hsg_status s = check_all(ens, n_ens, kState | kAnneal);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err;
        const hsg_ensemble e = launch_copy(ens[i]);
        if (hsg::resident_supported(e))
            err = hsg::launch_resident(e, 0, n_hb, n_or, 1, parity, 0, as_stream(stream));
        else
            err = hsg::launch_stream_anneal(e, parity, n_hb, n_or, 0, as_stream(stream));
        if (err != hipSuccess) return device(err, "anneal legs");
        err = hsg::launch_anneal_decide(ens[i], parity, as_stream(stream));
        if (err != hipSuccess) return device(err, "anneal decision");
    }
    return ok();
}

hsg_status hsg_decimate_swap(const hsg_ensemble* ens, int n_ens, int pairing, void* stream) {
    if (pairing < 0 || pairing > 2) return fail(HSG_ERR_INVALID, "pairing must be 0, 1 or 2 (got %d)", pairing);
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        if (ens[i].n_temps > 65536)
            return fail(HSG_ERR_UNSUPPORTED, "ensemble %d: n_temps > 65536", i);
        if (ens[i].work && !aligned(ens[i].work, 8))
            return fail(HSG_ERR_INVALID, "ensemble %d: work must be 8-byte aligned", i);
    }
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_decimate(ens[i], pairing, as_stream(stream));
        if (err != hipSuccess) return device(err, "decimated exchange");
    }
    return ok();
}

hsg_status hsg_coolheat_swap(const hsg_ensemble* ens, int n_ens, int pairing, double eps, void* stream) {
    if (pairing < 0 || pairing > 2) return fail(HSG_ERR_INVALID, "pairing must be 0, 1 or 2 (got %d)", pairing);
    if (!(eps >= 0.0) || !(eps < 1e6)) return fail(HSG_ERR_INVALID, "eps must be finite and >= 0 (got %g)", eps);
    hsg_status s = check_all(ens, n_ens, kState | kScratch);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i)
        if (!ens[i].work || !aligned(ens[i].work, 8))
            return fail(HSG_ERR_INVALID, "ensemble %d: work ([S][C][R-1][2] doubles) is required", i);
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_coolheat(ens[i], pairing, eps, nullptr, as_stream(stream));
        if (err != hipSuccess) return device(err, "cooling/heating exchange");
    }
    return ok();
}

hsg_status hsg_coolheat_swap_pairs(const hsg_ensemble* ens, int n_ens, int pairing, const double* eps,
                                   void* stream) {
    if (pairing < 0 || pairing > 2) return fail(HSG_ERR_INVALID, "pairing must be 0, 1 or 2 (got %d)", pairing);
    if (!eps || !aligned(eps, 8))
        return fail(HSG_ERR_INVALID, "eps must be a device array of doubles, 8-byte aligned");
    hsg_status s = check_all(ens, n_ens, kState | kScratch);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i)
        if (!ens[i].work || !aligned(ens[i].work, 8))
            return fail(HSG_ERR_INVALID, "ensemble %d: work ([S][C][R-1][2] doubles) is required", i);
    size_t off = 0;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_coolheat(ens[i], pairing, 0.0, eps + off, as_stream(stream));
        if (err != hipSuccess) return device(err, "cooling/heating exchange");
        off += static_cast<size_t>(ens[i].n_temps - 1);
    }
    return ok();
}

hsg_status hsg_measure(const hsg_ensemble* ens, int n_ens, void* stream) {
    hsg_status s = check_all(ens, n_ens, kState | kMeasure);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err = hsg::launch_measure(ens[i], as_stream(stream));
        if (err != hipSuccess) return device(err, "measure");
    }
    return ok();
}

hsg_status hsg_sweep_measure(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                             void* stream) {
    if (n_sweeps < 0 || n_hb < 0 || n_hb > 127 || n_or < 0 || n_hb + n_or < 1)
        return fail(HSG_ERR_INVALID, "need n_sweeps >= 0, 0 <= n_hb <= 127, n_or >= 0, n_hb + n_or >= 1 (got %d, %d, %d)",
                    n_sweeps, n_hb, n_or);
    hsg_status s = check_all(ens, n_ens, kState | kMeasure);
    if (s != HSG_OK) return s;
    for (int i = 0; i < n_ens; ++i) {
        if (!use_resident(ens[i], nullptr)) {
            s = check_one(ens[i], i, kScratch);
            if (s != HSG_OK) return s;
        }
    }
    for (int i = 0; i < n_ens; ++i) {
        hipError_t err;
        if (n_sweeps > 0 && hsg::resident_pair_supported(ens[i])) {
            err = hsg::launch_resident_pair(launch_copy(ens[i]), n_sweeps, n_hb, n_or, as_stream(stream));
            if (err != hipSuccess) return device(err, "sweep and measure");
            continue;
        }
        if (n_sweeps > 0 && hsg::resident_mseq_supported(ens[i])) {
            err = hsg::launch_resident_mseq(launch_copy(ens[i]), n_sweeps, n_hb, n_or, as_stream(stream));
            if (err != hipSuccess) return device(err, "sweep and measure");
            continue;
        }
        if (n_sweeps > 0 && !use_resident(ens[i], nullptr)) {
            // streaming sweeps: the measurement adds up the last sweep's per-tile
            // energies itself, in place of the sweep's own finishing pass
            int n_tiles = 0;
            err = hsg::launch_stream_sweeps(launch_copy(ens[i]), n_sweeps, n_hb, n_or, 0, 0, nullptr,
                                            as_stream(stream), true, &n_tiles);
            if (err != hipSuccess) return device(err, "sweep");
            err = hsg::launch_measure_fin(ens[i], n_tiles, n_sweeps, as_stream(stream));
            if (err != hipSuccess) return device(err, "measure");
            continue;
        }
        if (n_sweeps > 0) {
            s = hsg_sweep(&ens[i], 1, n_sweeps, n_hb, n_or, stream);
            if (s != HSG_OK) return s;
        }
        err = hsg::launch_measure(ens[i], as_stream(stream));
        if (err != hipSuccess) return device(err, "measure");
    }
    return ok();
}

hsg_status hsg_check(const hsg_ensemble* ens, int n_ens, void* stream) {
    hsg_status s = check_all(ens, n_ens, kState);
    if (s != HSG_OK) return s;
    hipError_t err = hipStreamSynchronize(as_stream(stream));
    if (err != hipSuccess) return device(err, "check: stream synchronize");
    for (int i = 0; i < n_ens; ++i) {
        int32_t g = 0;
        err = hipMemcpy(&g, ens[i].guard, sizeof(g), hipMemcpyDeviceToHost);
        if (err != hipSuccess) return device(err, "check: read guard");
        if (g != 0)
            return fail(HSG_ERR_NUMERIC, "ensemble %d: guard = %d (%s%s%s%s%s)", i, g,
                        (g & 1) ? "non-finite or non-unit spin or energy; " : "",
                        (g & 2) ? "protocol length outside [0, anneal_K_max]; " : "",
                        (g & 4) ? "temperature label outside [0, R); " : "",
                        (g & 8) ? "cooling map not a bijection (eps |S| >= 1); " : "",
                        (g & 16) ? "a wait of the persistent batch launch timed out (results invalid)" : "");
    }
    return ok();
}

static hsg_status mlp_check(int I, int H, int O, int B) {
    if (I < 1 || I > 64 || O < 1 || O > 64 || H < 1 || H > 256 || B < 0)
        return fail(HSG_ERR_INVALID, "MLP sizes out of range (I=%d H=%d O=%d B=%d)", I, H, O, B);
    return HSG_OK;
}

hsg_status hsg_mlp_forward(const float* params, int I, int H, int O, const float* x, int B,
                           float* acts, float* y, void* stream) {
    hsg_status s = mlp_check(I, H, O, B);
    if (s != HSG_OK) return s;
    if (!params || (B > 0 && (!x || !acts || !y))) return fail(HSG_ERR_INVALID, "MLP forward: NULL pointer");
    return device(hsg::launch_mlp_forward(params, I, H, O, x, B, acts, y, as_stream(stream)), "mlp_forward");
}

hsg_status hsg_mlp_backward(const float* params, int I, int H, int O, const float* x, int B,
                            float* acts, const float* dy, float* dparams, void* stream) {
    hsg_status s = mlp_check(I, H, O, B);
    if (s != HSG_OK) return s;
    if (!params || !dparams || (B > 0 && (!x || !acts || !dy)))
        return fail(HSG_ERR_INVALID, "MLP backward: NULL pointer");
    return device(hsg::launch_mlp_backward(params, I, H, O, x, B, acts, dy, dparams, as_stream(stream)),
                  "mlp_backward");
}

hsg_status hsg_mlp_mse_grad(const float* y, const float* t, const float* w, int B, int O,
                            float* dy, double* loss, void* stream) {
    if (B < 0 || O < 1 || O > 64 || (B > 0 && (!y || !t || !dy)))
        return fail(HSG_ERR_INVALID, "MLP mse_grad: bad arguments");
    if (B == 0) return ok();
    return device(hsg::launch_mlp_mse_grad(y, t, w, B, O, dy, loss, as_stream(stream)), "mlp_mse_grad");
}

hsg_status hsg_mlp_adam(float* params, const float* grad, float* m, float* v, int n, float lr,
                        float beta1, float beta2, float eps, int t, void* stream) {
    if (!params || !grad || !m || !v || n < 0 || t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(HSG_ERR_INVALID, "MLP adam: bad arguments");
    if (n == 0) return ok();
    return device(hsg::launch_mlp_adam(params, grad, m, v, n, lr, beta1, beta2, eps, t, as_stream(stream)),
                  "mlp_adam");
}

hsg_status hsg_probe_issue(int kind, int n_groups, int group_threads, int iters, float* sink, void* stream) {
    if (kind < 0 || kind > 4) return fail(HSG_ERR_INVALID, "probe: kind %d outside [0, 4]", kind);
    if (n_groups < 1 || n_groups > (1 << 20) || group_threads < 64 || group_threads > 1024 ||
        group_threads % 64 != 0 || iters < 1)
        return fail(HSG_ERR_INVALID, "probe: need 1 <= n_groups <= 2^20, group_threads a multiple of 64 "
                                     "in [64, 1024], iters >= 1 (got %d, %d, %d)",
                    n_groups, group_threads, iters);
    if (!sink || !aligned(sink, 4)) return fail(HSG_ERR_INVALID, "probe: sink is NULL or misaligned");
    return device(hsg::launch_probe_issue(kind, n_groups, group_threads, iters, sink, as_stream(stream)),
                  "probe_issue");
}

}  // extern "C"
