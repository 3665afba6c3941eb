// Internal launcher interface between the C ABI (abi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hsgpt.h"

namespace hsg {

// The thread's message for hsg_last_error (entry points implemented outside abi.hip).
void set_last_error(const char* msg);

// Largest dynamic LDS a workgroup may use on this device (bytes).
size_t max_block_lds();
// Allows `kern` more than 64 KiB of dynamic LDS on the current device (once per
// kernel and device; thread-safe).
hipError_t allow_dynamic_lds(const void* kern, size_t lds);

// Compute units of the current device, and how many workgroups of `kern` (nt
// threads, lds bytes of dynamic LDS) one CU holds (queried once per kernel and device).
int device_cus();
hipError_t blocks_per_cu_query(const void* kern, int nt, size_t lds, int* out);

// One persistent launch over the regular sweeps of all the ensembles of a call (at most
// 8, one precision; L >= 4; ensembles swept in tiles and the first one need their
// scratch): L = 12..16 classes in LDS from a work counter, the others half-sweep by
// half-sweep behind a barrier of their own partition of `g_str` workgroups (0: by the
// classes' share of the work).
bool batch_supported(const hsg_ensemble* ens, int n_ens);
bool batch_needs_scratch(const hsg_ensemble& e);
hipError_t launch_batch_sweeps(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or, int g_str,
                               hipStream_t st);

// LDS-resident path: true if one replica of `e` fits in a workgroup's LDS and
// an instantiation for e.L exists.
bool resident_supported(const hsg_ensemble& e);
// ... and twice that fits (the two replica buffers of the persistent
// double-buffered workgroups).
bool persistent_supported(const hsg_ensemble& e);
// The persistent single-buffer workgroups (k_resident_chain): binary32, L = 16.
bool chain_supported(const hsg_ensemble& e);
// Regular sweeps, one workgroup per replica (anneal = 0), the annealing legs of
// one parity (anneal = 1), or regular sweeps on persistent double-buffered
// workgroups (anneal = 2) or on persistent single-buffer ones (anneal = 3).
hipError_t launch_resident(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, int anneal,
                           int parity, int block_threads, hipStream_t st);

// Regular sweeps of both chains' replicas at one temperature per workgroup followed
// by the measurement of that temperature (the results of launch_resident with
// anneal = 0 and then launch_measure): ensembles of exactly two chains at the sizes
// where this one launch is faster (binary32 L <= 10, binary64 L <= 12).
bool resident_pair_supported(const hsg_ensemble& e);
// One workgroup per (sample, temperature) sweeping the chain-0 then the chain-1 replica
// and measuring the pair (binary32, L = 16, two chains): the results of launch_resident
// with anneal = 0 and launch_measure, Q and chi within rounding.
bool resident_mseq_supported(const hsg_ensemble& e);
hipError_t launch_resident_mseq(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st);
hipError_t launch_resident_pair(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st);

// Wavefront path: one workgroup per replica walking its z-planes, one HBM pass per
// lattice sweep (L = 18 .. 40 in binary32, .. 28 in binary64, LDS permitting); a
// tuning option, slower than the streaming path where measured.
bool wave_supported(const hsg_ensemble& e);
hipError_t launch_wave_sweeps(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or, hipStream_t st);

// Streaming path: one launch per half-sweep, any even L.  The per-tile energy sums go
// to `partial` ([slots][max_tiles] doubles), or to the ensemble's scratch if null.
// defer_last: the last sweep's per-tile sums are left for launch_measure_fin to add up
// (energies, sweep counters), which then must follow on the same stream; *n_tiles_out
// (if given) receives the tiles per slot.
hipError_t launch_stream_sweeps(const hsg_ensemble& e, int n_sweeps, int n_hb, int n_or,
                                int block_threads, int replicas_per_block, double* partial,
                                hipStream_t st, bool defer_last = false, int* n_tiles_out = nullptr);
// Capacity (doubles) of the library's own device array that serves as `partial` for
// callers that cannot allocate, and its address on the current device.
constexpr size_t kStaticPartialDoubles = size_t(1) << 19;  // 4 MiB
hipError_t static_partial(double** out);
hipError_t launch_stream_anneal(const hsg_ensemble& e, int parity, int n_hb, int n_or,
                                int block_threads, hipStream_t st);

// Initialisation, energy, exchange, measurement.
hipError_t launch_init_couplings(const hsg_ensemble& e, hipStream_t st);
hipError_t launch_init_spins(const hsg_ensemble& e, int cold, hipStream_t st);
hipError_t launch_energy(const hsg_ensemble& e, double* out, hipStream_t st);
hipError_t launch_swap(const hsg_ensemble& e, int pairing, hipStream_t st);
hipError_t launch_anneal_decide(const hsg_ensemble& e, int parity, hipStream_t st);
hipError_t launch_measure(const hsg_ensemble& e, hipStream_t st);
// The measurement that also finishes a streaming sweep launched with defer_last: each
// slot's energy from its n_tiles per-tile sums in the scratch (in tile order, as the
// sweep's own finishing pass adds them), and sweep_ctr += ctr_add.
hipError_t launch_measure_fin(const hsg_ensemble& e, int n_tiles, int ctr_add, hipStream_t st);
hipError_t launch_decimate(const hsg_ensemble& e, int pairing, hipStream_t st);
// eps_pair: nullptr (eps for every pair) or a device array of n_temps - 1 parameters.
hipError_t launch_coolheat(const hsg_ensemble& e, int pairing, double eps, const double* eps_pair, hipStream_t st);

// MLP
hipError_t launch_mlp_forward(const float* p, int I, int H, int O, const float* x, int B,
                              float* acts, float* y, hipStream_t st);
hipError_t launch_mlp_backward(const float* p, int I, int H, int O, const float* x, int B,
                               float* acts, const float* dy, float* dp, hipStream_t st);
hipError_t launch_mlp_mse_grad(const float* y, const float* t, const float* w, int B, int O, float* dy,
                               double* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr,
                           float b1, float b2, float eps, int t, hipStream_t st);

// issue-rate probe (probe.hip); arguments checked by the caller
hipError_t launch_probe_issue(int kind, int n_groups, int threads, int iters, float* sink, hipStream_t st);

}  // namespace hsg
