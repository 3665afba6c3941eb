/*
 * hsgref -- plain FP64 CPU oracle for the parallel-tempering hot path of the
 * three-dimensional Heisenberg spin glass (Hasenbusch & Schaefer, "Speeding up
 * parallel tempering simulations", arXiv:1006.4247).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU library and the GPU library never
 * calls it.
 *
 * Natural layouts (host arrays, all double precision):
 *   site index      x = i + L*(j + L*k), 0 <= i,j,k < L, periodic
 *   couplings J     [S][N][3]      J[x][mu] couples x and x + e_mu
 *   spins           [S][C][R][N][3] indexed by slot (a physical configuration)
 *   per-slot arrays [S][C][R]; per-chain arrays [S][C]; per-pair [S][C][R-1]
 */
#ifndef HSGREF_H
#define HSGREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* counter-based generator and uniform maps */
void   hsgref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double hsgref_u01_24(uint32_t w);
double hsgref_u01_52(uint32_t w0, uint32_t w1);

/* lattice */
int  hsgref_parity(int L, int x);
int  hsgref_compressed_index(int L, int x);
int  hsgref_neighbor(int L, int x, int dir); /* dir: 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z */

/* initialisation */
void hsgref_init_couplings(int L, int n_samples, uint32_t sample_base, uint64_t seed,
                           int round_f32, double* J);
void hsgref_init_spins(int L, int n_slots, uint32_t slot_base, uint64_t seed,
                       int cold, int round_f32, double* s);

/* single-site pieces */
void   hsgref_local_field(int L, const double* J, const double* s, int x, double S[3]);
void   hsgref_heatbath_spin(const double S[3], double beta, double r1, double r2, double out[3]);
void   hsgref_overrelax_spin(const double s[3], const double S[3], double out[3]);
void   hsgref_fields(int L, const double* J, const double* s, int parity, double* S_out);
void   hsgref_hb_uniforms_all(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t t,
                              uint32_t hs, int parity, double* r1, double* r2);
void   hsgref_heatbath_many(int n, const double* S, const double* beta, const double* r1,
                            const double* r2, double* out);
void   hsgref_overrelax_many(int n, const double* s, const double* S, double* out);
void   hsgref_hb_uniforms(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t t,
                          uint32_t hs, int x, double* r1, double* r2);

/* energies of one replica */
double hsgref_energy(int L, const double* J, const double* s);
double hsgref_sublattice_energy(int L, const double* J, const double* s, int parity);

/* one replica: half-sweep and sweep */
void hsgref_halfsweep(int L, const double* J, double* s, int parity, int kind, double beta,
                      uint64_t seed, uint32_t slot_global, uint32_t t, uint32_t hs, int rng32,
                      const int32_t* order);
void hsgref_sweep(int L, const double* J, double* s, int n_hb, int n_or, int adjoint,
                  double beta, uint64_t seed, uint32_t slot_global, uint32_t t, int rng32);

/* ensembles */
void hsgref_sweep_batch(int L, int S, int C, int R, const double* J, double* spins,
                        const double* betas, const int32_t* temp_of_slot, uint32_t* sweep_ctr,
                        uint32_t slot_base, uint64_t seed, int n_sweeps, int n_hb, int n_or,
                        int rng32, double* energy);
void hsgref_swap_batch(int S, int C, int R, const double* betas, const double* energy,
                       int32_t* temp_of_slot, int32_t* slot_of_temp, uint32_t* swap_ctr,
                       int64_t* stats, int32_t* rt_state, int64_t* rt_trips,
                       uint32_t chain_base, uint64_t seed, int pairing);
void hsgref_anneal_batch(int L, int S, int C, int R, const double* J, double* spins,
                         const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                         uint32_t* sweep_ctr, uint32_t* swap_ctr, double* energy,
                         int64_t* stats, int32_t* rt_state, int64_t* rt_trips,
                         uint32_t slot_base, uint32_t chain_base, uint64_t seed, int parity,
                         const int32_t* K, const double* lambda, int K_max, int n_hb, int n_or,
                         int rng32, double* work_out);
double hsgref_log_sinhc(double u);
double hsgref_decimated_log_ratio(int L, const double* J, const double* sx, const double* sy,
                                  int d, double b1, double b2);
void hsgref_decimate_uniforms(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t n,
                              uint32_t pair, int x, double* r1, double* r2);
int hsgref_decimate_role(uint64_t seed, uint32_t chain_global, uint32_t n);
void hsgref_decimate_batch(int L, int S, int C, int R, const double* J, double* spins,
                           const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                           uint32_t* swap_ctr, double* energy, int64_t* stats, int32_t* rt_state,
                           int64_t* rt_trips, uint32_t slot_base, uint32_t chain_base,
                           uint64_t seed, int pairing, int rng32, double* log_ratio_out,
                           int32_t* role_out);
double hsgref_cool_spin(const double s[3], const double S[3], double eps, double out[3]);
double hsgref_heat_spin(const double sp[3], const double S[3], double eps, double out[3]);
double hsgref_coolheat(int L, const double* J, double* s, double eps, int heat);
void hsgref_coolheat_batch(int L, int S, int C, int R, const double* J, double* spins,
                           const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                           uint32_t* swap_ctr, double* energy, int64_t* stats, int32_t* rt_state,
                           int64_t* rt_trips, uint32_t chain_base, uint64_t seed, int pairing,
                           double eps, double* log_ratio_out, double* logdet_out,
                           const double* eps_pair);
void hsgref_measure_batch(int L, int S, int C, int R, const double* spins, const double* energy,
                          const int32_t* slot_of_temp, double* Q, double* chi, double* e);
void hsgref_roundtrip_update(int R, const int32_t* temp_of_slot, int32_t* rt_state,
                             int64_t* rt_trips);
int  hsgref_num_threads(void);
/* Threads of the parallel loops from now on (n >= 1). */
void hsgref_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
