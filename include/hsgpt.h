/*
 * hsgpt.h -- C ABI of the MI355X (gfx950) library for the parallel-tempering hot
 * path of the three-dimensional Heisenberg spin glass, the method studied in
 * Hasenbusch & Schaefer, "Speeding up parallel tempering simulations"
 * (arXiv:1006.4247).
 *
 * Model (paper Sec. I, Eq. (2)): O(3) unit spins s_x on an L^3 periodic simple
 * cubic lattice, H = -sum_<xy> J_xy s_x.s_y with quenched Gaussian J_xy.
 *
 * General conventions
 *  - Every pointer inside hsg_ensemble is a DEVICE pointer owned by the caller;
 *    the library never allocates, frees or retains caller memory.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL = the default stream) except hsg_check, which synchronises it.
 *  - Argument errors are found before any launch: the call returns
 *    HSG_ERR_INVALID and hsg_last_error() says why; nothing was enqueued.
 *  - A launch failure returns HSG_ERR_DEVICE with the HIP error string.
 *  - Numerical trouble seen by a kernel (a non-finite spin or energy, a spin
 *    whose norm left 1 by more than the precision's tolerance, a protocol
 *    length outside [0, anneal_K_max], a temperature label outside [0, R), a
 *    cooling map that is not a bijection, a wait of the persistent batch launch that
 *    ran out) is latched in *guard (bits 1, 2, 4, 8, 16)
 *    and reported by hsg_check as
 *    HSG_ERR_NUMERIC.  Out-of-range values are clamped before use, so a
 *    corrupted label or protocol length never addresses outside its ensemble.
 *  - Calls on one ensemble must not overlap in time (use one stream per
 *    ensemble); distinct ensembles may be driven from distinct threads.
 *
 * Lattice and layouts
 *  - site x = i + L(j + L k), 0 <= i,j,k < L; L even, 2 <= L <= 64.
 *  - parity p(x) = (i+j+k) mod 2: p = 0 is the white sublattice W, p = 1 the
 *    black one B (paper Sec. III.A).  Index inside a sublattice:
 *    h = floor(i/2) + (L/2)(j + L k), 0 <= h < N/2, N = L^3.
 *  - spins:      [S][C][R][3][2][N/2] of T (component, parity, h); T = double
 *                (HSG_FP64) or float (HSG_FP32).  Slot r of chain c of sample s
 *                holds one physical configuration.
 *  - couplings:  [S][3][2][N/2] of T: J(x, mu) joins x and x + e_mu, stored at
 *                the parity and index of x.
 *  - betas:      [R] double, strictly ascending (not checked).
 *  - per slot:   temp_of_slot, rt_state int32, energy double, sweep_ctr uint32,
 *                rt_trips int64, all [S][C][R]; slot_of_temp int32 [S][C][R]
 *                is indexed by temperature.
 *  - per chain:  swap_ctr uint32 [S][C]; per pair: swap_stats int64
 *                [S][C][R-1][2] (attempts, accepts).
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed
 * (low word, high word); counters (c0, c1, c2, c3):
 *    couplings (x, mu, sample_base + s, 1<<24)
 *    spin init (x, 0, slot_g, 2<<24)
 *    heat-bath (h or h mod N/4, sweep_ctr[slot], slot_g, 3<<24 | hs<<16)
 *    exchange  (pair i, swap_ctr[chain], chain_base + s C + c, 4<<24)
 * with slot_g = slot_base + (s C + c) R + r and hs = 2*(heat-bath sweep) + parity.
 * 52-bit uniforms ((w0<<20 | w1>>12) + 1/2) 2^-52 serve FP64 and all
 * initialisation and exchange decisions; FP32 heat-bath uses 23-bit uniforms
 * ((w>>9) + 1/2) 2^-23, one block per site pair (h, h + N/4).
 */
#ifndef HSGPT_H
#define HSGPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSG_ABI_VERSION 1

typedef enum {
    HSG_OK = 0,
    HSG_ERR_INVALID = 1,
    HSG_ERR_DEVICE = 2,
    HSG_ERR_NUMERIC = 3,
    HSG_ERR_UNSUPPORTED = 4
} hsg_status;

typedef enum { HSG_FP64 = 0, HSG_FP32 = 1 } hsg_precision;

/* One size class: S samples (coupling sets) x C chains x R temperatures. */
typedef struct hsg_ensemble {
    int32_t L, n_samples, n_chains, n_temps;
    int32_t precision; /* hsg_precision */
    int32_t reserved0; /* ignored (the library sets it in its own copies) */
    uint32_t sample_base, chain_base, slot_base; /* global stream offsets */
    uint32_t reserved1;
    uint64_t seed;
    /* state */
    void* spins;
    void* couplings;
    const double* betas;
    int32_t* temp_of_slot;
    int32_t* slot_of_temp;
    double* energy;
    uint32_t* sweep_ctr;
    uint32_t* swap_ctr;
    int64_t* swap_stats;
    int32_t* rt_state;
    int64_t* rt_trips;
    int32_t* guard;
    /* annealed exchange (may be NULL unless hsg_anneal_swap is called) */
    const int32_t* anneal_K;      /* [R-1] protocol lengths, 0..anneal_K_max */
    const double* anneal_lambda;  /* [R-1][anneal_K_max] interior betas, or NULL = linear */
    int32_t anneal_K_max;
    int32_t reserved2;
    void* scratch;                /* hsg_scratch_bytes() bytes, 256-byte aligned: needed by
                                     hsg_anneal_swap and by sweeps on the streaming path */
    double* work;                 /* [S][C][R-1][2] W_up, W_down of the last call */
    /* measurement outputs (may be NULL unless hsg_measure is called) */
    double* Q;      /* [S][R][3][3] */
    double* chi;    /* [S][R]       */
    double* e_temp; /* [S][C][R]    */
} hsg_ensemble;

/* Tuning knobs of the sweep kernels (0 = library default). */
typedef struct hsg_tuning {
    int32_t path;           /* 0 auto (3 if a replica fits in one workgroup's LDS, else 2);
                               1 LDS-resident lattice on persistent double-buffered
                               workgroups; 2 streaming half-sweeps; 3 LDS-resident lattice,
                               one workgroup per replica; 4 wavefront: one workgroup per
                               replica walking its z-planes, one HBM pass per lattice
                               sweep (L 18..40 binary32, 18..28 binary64); 5 one persistent
                               launch over all the ensembles of the call (at most 8, one
                               precision, L >= 4): L = 12, 14, 16 swept in LDS, one
                               replica per work item from a counter, the others in tiles
                               half-sweep by half-sweep behind a barrier of their own
                               part of the grid (they, and the first ensemble, need their
                               scratch); spins as with the other paths, bit for bit;
                               6 LDS-resident lattice on persistent single-buffer
                               workgroups, each sweeping a contiguous range of replicas
                               with the next one's loads in flight (binary32, L = 16;
                               spins and energies as with path 3, bit for bit) */
    int32_t block_threads;  /* threads per workgroup (path 5: workgroups of the tiled part,
                               a multiple of 8; 0 = by its share of the work) */
    int32_t replicas_per_block; /* streaming path: replicas sharing one coupling tile */
    int32_t flags;          /* HSG_TUNE_NO_RENORM: binary32 sweeps without a heat-bath lattice
                               sweep skip their once-per-sweep renormalisation s <- s/|s|
                               (on by default; it keeps |s| = 1 under reflections alone) */
} hsg_tuning;

#define HSG_TUNE_NO_RENORM 1

int hsg_abi_version(void);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* hsg_last_error(void);

/* Bytes of device scratch one ensemble needs for hsg_anneal_swap. */
size_t hsg_scratch_bytes(const hsg_ensemble* ens);

/* Draw J_xy ~ N(0,1) for every sample (paper Sec. I: Gaussian couplings of zero
 * mean and unit width), Box-Muller cosine branch from two 52-bit uniforms,
 * computed in FP64 and rounded to T. */
hsg_status hsg_init_couplings(const hsg_ensemble* ens, int n_ens, void* stream);

/* Start every slot: uniform unit spins (z = 2 r1 - 1, azimuth 2 pi r2), or the
 * cold start (1,0,0) of the paper's Sec. IV.C if cold != 0.  Resets labels to
 * the identity, counters, statistics, round-trip state (slot 0 starts at the
 * highest temperature) and the guard, and computes every slot's energy. */
hsg_status hsg_init_spins(const hsg_ensemble* ens, int n_ens, int cold, void* stream);

/* n_sweeps sweeps of every slot at its own temperature betas[temp_of_slot].
 * One sweep = n_hb heat-bath lattice sweeps then n_or overrelaxation lattice
 * sweeps, each as the W then the B half-sweep (paper Sec. III.C; checkerboard
 * order instead of the paper's typewriter order, same stationary law).
 * Heat-bath: new spin along S_x with density ~ exp(beta S_x.s); overrelaxation:
 * s' = 2 (s.S)/S^2 S - s (identity if S = 0).  Leaves energy[] = H of the
 * final configurations (fused into the last half-sweep) and advances
 * sweep_ctr by n_sweeps.  n_sweeps >= 0, n_hb in [0,127], n_or >= 0. */
hsg_status hsg_sweep(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                     void* stream);
hsg_status hsg_sweep_tuned(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb,
                           int n_or, const hsg_tuning* tuning, void* stream);

/* hsg_sweep for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same sweeps,
 * results bit for bit those of hsg_sweep with the default tuning, without
 * ens[i].scratch (it may be NULL).  Ensembles on the streaming path (those whose
 * replica does not fit one workgroup's LDS) keep their per-tile energy sums in a
 * device array of the library's own, 4 MiB per device (held until the process ends;
 * 4 MiB = 524288 doubles, enough for slots x ceil(L^3/256) doubles: e.g. 512 slots
 * at L = 32, 37 slots at L = 64); a larger ensemble returns HSG_ERR_INVALID before
 * anything is enqueued.  Nothing is allocated.  Every call on one device shares
 * that array, so calls on one device that overlap in time (different streams or host
 * threads) race and must be serialised by the caller; consecutive calls on one
 * stream are safe (each sum is written before it is read). */
hsg_status hsg_sweep_static(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                            void* stream);

/* H = -sum over bonds J s.s (Eq. (2)) of every slot, from scratch, in FP64.
 * H_out: device array of sum_e S_e C_e R_e doubles, ensembles in order, slot
 * layout [S][C][R]; NULL writes ens[e].energy instead. */
hsg_status hsg_energy(const hsg_ensemble* ens, int n_ens, double* H_out, void* stream);

/* Replica exchange, Eq. (1): for each selected pair i of every chain the
 * configurations at beta_i and beta_{i+1} exchange temperature labels iff
 * ln u < (beta_{i+1} - beta_i)(H_{i+1} - H_i).  pairing 0: all pairs in
 * ascending order; 1: even i; 2: odd i.  Updates labels, swap_stats,
 * round-trip state (paper Sec. IV.B) and swap_ctr. */
hsg_status hsg_swap(const hsg_ensemble* ens, int n_ens, int pairing, void* stream);

/* Annealed exchange of the pairs i with i mod 2 == parity (a nonequilibrium-
 * switch exchange, the prior art the paper cites in Sec. I).  With
 * a = beta_i < l_1 < ... < l_K < b = beta_{i+1} (K = anneal_K[i]; l_k from
 * anneal_lambda or linear), the configuration x at a takes K sweeps at
 * l_1..l_K in forward order and y at b takes K sweeps at l_K..l_1 in adjoint
 * (reversed) order, each sweep of n_hb heat-bath and n_or overrelaxation
 * lattice sweeps; W_up = sum_k (l_{k+1}-l_k) H(x_k), W_dn likewise downwards.
 * Accept iff ln u < -(W_up + W_dn): the annealed states take the exchanged
 * temperatures; otherwise both configurations keep their states.  K = 0 is
 * Eq. (1) exactly.  Needs anneal_K, scratch (hsg_scratch_bytes) and work. */
hsg_status hsg_anneal_swap(const hsg_ensemble* ens, int n_ens, int parity, int n_hb, int n_or,
                           void* stream);

/* Decimated replica exchange (paper Sec. III.A, Eq. (eq:aswap)) of the selected
 * pairs of every chain (pairing 0: all pairs in ascending order; 1: even i;
 * 2: odd i).  Pair i decimates sublattice D_i = (d_0 + i) mod 2 (parity of
 * i + j + k), d_0 one random bit per chain and call.  With S_z the local field
 * of the kept sublattice at z in D and h(u) = ln(sinh(u)/u),
 *   ln A = sum_{z in D} h(b2 |S_z(x)|) - h(b1 |S_z(x)|) + h(b1 |S_z(y)|) - h(b2 |S_z(y)|)
 * for x at b1 = beta_i and y at b2 = beta_{i+1}, in FP64 (fields in the spin
 * precision).  Accept iff ln u < ln A (u from the same per-pair stream as
 * hsg_swap): the labels are exchanged and the D spins of x and y are drawn anew
 * by heat-bath at beta_{i+1} and beta_i, and their energies recomputed;
 * otherwise nothing changes.  Advances swap_ctr, updates swap_stats and round
 * trips.  If work is not NULL it receives, per pair, ln A and D_i
 * ([S][C][R-1][2]; 0 and -1 for pairs not attempted).  n_temps <= 65536. */
hsg_status hsg_decimate_swap(const hsg_ensemble* ens, int n_ens, int pairing, void* stream);

/* Cooling / heating replica exchange (paper Sec. III.B) of the selected pairs of
 * every chain (pairing 0: all pairs in ascending order, each seeing the states
 * the previous pair left; 1: even i; 2: odd i).  Site map with field S of the
 * other sublattice, k = eps |S|, cos(theta) = s.S/|S|: cooling turns s towards S
 * by alpha = k sin(theta) in the plane of s and S; heating is its inverse
 * (Newton's method on theta - k sin(theta) = theta').  The lattice cooling C maps
 * sublattice 0 and then 1; C^-1 undoes 1 and then 0.  For x at b1 = beta_i and
 * y at b2 = beta_{i+1} the involution (x, y) -> (C^-1 y at b1, C x at b2) is
 * accepted iff ln u < ln A,
 *   ln A = b1 H(x) + b2 H(y) - b1 H(C^-1 y) - b2 H(C x)
 *          + ln det J_C(x) - ln det J_C(C^-1 y)
 * (FP64; maps in the spin precision; u from the same per-pair stream as
 * hsg_swap); eps = 0 is Eq. (1).  Accepted pairs take the transformed states at
 * the exchanged temperatures, rejected pairs change nothing.  A site with
 * eps |S| >= 1 (the map is then not a bijection) rejects its pair and sets guard
 * bit 8.  Needs scratch (hsg_scratch_bytes) and work, which receives
 * ln det J_C(x) and ln det J_C(C^-1 y) per pair ([S][C][R-1][2], zeros for the
 * pairs not attempted).  Advances swap_ctr, updates swap_stats and round trips. */
hsg_status hsg_coolheat_swap(const hsg_ensemble* ens, int n_ens, int pairing, double eps,
                             void* stream);

/* hsg_coolheat_swap with one map parameter per pair of temperatures (paper Sec. IV
 * suggests tuning eps for each pair of beta values separately): pair i of ensemble e
 * uses eps[o_e + i], o_e = sum over the ensembles before e of (n_temps - 1).  eps:
 * device array of doubles, 8-byte aligned, owned by the caller; values must be
 * finite and >= 0 (a value with eps |S| >= 1 at some site rejects that pair and sets
 * guard bit 8, as above; other values are not checked on the host).  Same needs and
 * outputs as hsg_coolheat_swap; equal values give its results bit for bit. */
hsg_status hsg_coolheat_swap_pairs(const hsg_ensemble* ens, int n_ens, int pairing, const double* eps,
                                   void* stream);

/* Overlap (paper Sec. II): Q_ab = sum_x s^(0)_{a,x} s^(1)_{b,x} between the
 * chain-0 and chain-1 configurations at each temperature, chi = Q:Q / N, and
 * e_temp = H/N by temperature (the paper's E is -e).  Q and chi need C >= 2. */
hsg_status hsg_measure(const hsg_ensemble* ens, int n_ens, void* stream);

/* hsg_sweep(ens, n_ens, n_sweeps, n_hb, n_or) followed by hsg_measure(ens, n_ens):
 * the same spins and counters, and the same energies and measurements up to the
 * rounding order of their FP64 sums.  Ensembles of exactly two chains with L <= 10
 * (binary32) or L <= 12 (binary64) take one launch, in which a workgroup sweeps both
 * chains' replicas of a temperature and measures them from LDS (measured faster
 * there); binary32 ones at L = 16 take one launch in which a workgroup sweeps the two
 * replicas of a temperature in turn, the couplings loaded once, and then measures
 * them.  On the streaming path (lattices whose replica does not fit one workgroup's
 * LDS) the measurement also adds up the last sweep's per-tile energies, in place of
 * the sweep's own finishing launch, in the same order (energies and counters bit for
 * bit those of hsg_sweep).  Other ensembles take the two calls.  Needs what both
 * calls need; n_sweeps = 0 measures only. */
hsg_status hsg_sweep_measure(const hsg_ensemble* ens, int n_ens, int n_sweeps, int n_hb, int n_or,
                             void* stream);

/* --- plans: a captured cycle of several ensembles ----------------------------
 * One cycle of the method (scope: the workloads' step) for every ensemble: n_hb
 * heat-bath and n_or overrelaxation lattice sweeps with the measurement of the swept
 * configurations (hsg_sweep_measure, or hsg_sweep_tuned + hsg_measure when a tuning is
 * given), then one exchange pass (hsg_swap, hsg_anneal_swap, hsg_decimate_swap or
 * hsg_coolheat_swap[_pairs]).  hsg_plan_create captures that cycle into HIP graphs
 * inside the library, each ensemble on a capture stream of its own so that the size
 * classes of an uneven batch run concurrently; hsg_plan_run launches it n_cycles
 * times on `stream` (one graph launch per cycle), with the results of the same calls
 * made eagerly, bit for bit.  Exchanges that alternate between even and odd pairs
 * (pairing -1; the annealed exchange always does) start with the even pairs and the
 * plan remembers the next parity across runs.
 *
 * tuning_json: NULL, "" or a flat JSON object; keys (all optional):
 *   "exchange": "plain" (default) | "anneal" | "decimate" | "coolheat" | "none"
 *   "pairing": -1 alternate even / odd pairs, 0 all ascending, 1 even, 2 odd
 *              (default 0 for plain, -1 otherwise)
 *   "n_hb", "n_or": sweep composition (default 1, 3); "measure": 0 | 1 (default 1)
 *   "anneal_n_hb", "anneal_n_or": composition of the annealing legs' sweeps
 *   "eps": one cooling / heating parameter, or an array of one per pair of every
 *          ensemble, ensembles in order (the library keeps its own device copy)
 *   "path", "block_threads", "replicas_per_block", "flags": hsg_tuning fields, one
 *          value or an array with one per ensemble
 *   "streams": 0 to capture all ensembles on one stream (default 1)
 *   "stream": one capture-stream index in [0, n_ens) per ensemble: ensembles with the
 *             same index run one after another on one stream, the streams side by side
 *             (default: a stream per ensemble); not with "split"
 *   "split": k in [1, 16] (default 1): each ensemble of at least two samples runs as k
 *            parts of consecutive samples, each on a capture stream of its own, so that
 *            one part's exchange and launch edges overlap another's sweep; results are
 *            those of the whole ensemble bit for bit.  Needs LDS-resident sweeps
 *            (L <= 16, path 0, 3 or 6); for the exchanges that use scratch the plan
 *            allocates the parts' scratch itself (hsg_scratch_bytes of each part)
 *   "unroll": the plan holds graphs of 1, 2, 4, ... cycles up to the largest power of
 *             two <= unroll (default 16); a run of n cycles launches the longest graphs
 *             that fit, at most about log2(n) launches, so that a graph launch (after
 *             which the streams drain) is paid once per many cycles
 * Unknown keys and malformed values are refused (HSG_ERR_INVALID).  The plan copies the
 * descriptors: the caller's device buffers must stay allocated, and the descriptors'
 * pointers unchanged, until hsg_plan_destroy.  Creating a plan enqueues nothing on the
 * caller's streams and changes no state; it allocates the graphs (and the per-pair eps
 * copy, and the split parts' scratch).  A plan is used from one host thread at a time,
 * on the device it was created on; runs on one plan must not overlap.  *plan receives
 * an opaque handle. */
hsg_status hsg_plan_create(const hsg_ensemble* ens, int n_ens, const char* tuning_json, void** plan);
hsg_status hsg_plan_run(void* plan, int n_cycles, void* stream);
hsg_status hsg_plan_destroy(void* plan);
/* Parity (0 even, 1 odd) of the next cycle's exchange (alternating plans; 0 otherwise),
 * and setting it (e.g. to continue a run that started eagerly). */
int hsg_plan_next_parity(const void* plan);
hsg_status hsg_plan_set_next_parity(void* plan, int parity);

/* Synchronise `stream`, then report the guards: HSG_ERR_NUMERIC if any is set. */
hsg_status hsg_check(const hsg_ensemble* ens, int n_ens, void* stream);

/* --- learned annealing schedule: a 2-hidden-layer MLP (FP32) ---------------
 * Layout of `params` (floats): W1[H][I], b1[H], W2[H][H], b2[H], W3[O][H], b3[O]
 * with tanh hidden activations and a linear output.  x: [B][I], y: [B][O];
 * 1 <= I, O <= 64, 1 <= H <= 256.  `acts` ([B][4H] floats, caller-owned) keeps
 * the two hidden activations (written by the forward pass) and the two layer
 * errors (written by the backward pass).  The backward pass reads dy [B][O]
 * (dLoss/dy per sample) and overwrites dparams (same layout as params) with
 * the gradient summed over the batch in a fixed order.  Adam: m, v same layout
 * as params; step t >= 1 (bias correction). */
hsg_status hsg_mlp_forward(const float* params, int I, int H, int O, const float* x, int B,
                           float* acts, float* y, void* stream);
hsg_status hsg_mlp_backward(const float* params, int I, int H, int O, const float* x, int B,
                            float* acts, const float* dy, float* dparams, void* stream);
/* Weighted squared error of the learner's surrogate fit: with y, t [B][O] and
 * optional sample weights w [B] (NULL = 1), writes dy = 2 w (y - t) / B and, if
 * loss != NULL, *loss = sum_b w_b sum_o (y - t)^2 / B (FP64, fixed summation order). */
hsg_status hsg_mlp_mse_grad(const float* y, const float* t, const float* w, int B, int O,
                            float* dy, double* loss, void* stream);
hsg_status hsg_mlp_adam(float* params, const float* grad, float* m, float* v, int n, float lr,
                        float beta1, float beta2, float eps, int t, void* stream);

/* --- diagnostics: issue rates of the compute units ----------------------------
 * The measured basis of the roofline peaks (the VALU and LDS rates the sweep kernels
 * are held against).  Launches n_groups workgroups of group_threads threads (a
 * multiple of 64 in [64, 1024]; 1 <= n_groups <= 2^20) on `stream`; every thread runs
 * `iters` >= 1 rounds of 16 independent operations of one kind: 0 binary32 FMA,
 * 1 binary64 FMA, 2 binary32 exp2 (a transcendental), 3 LDS reads of 4-byte words,
 * 4 LDS reads of 16-byte vectors (kinds 3 and 4: each wave reads consecutive
 * addresses, 64 bytes per thread per round).  `sink` (device, caller-owned,
 * n_groups * group_threads floats) receives one value per thread, so that no work is
 * optimised away.  The caller times the launch on `stream`: lane-operations =
 * n_groups * group_threads * iters * 16.  Reads nothing else and keeps no state. */
hsg_status hsg_probe_issue(int kind, int n_groups, int group_threads, int iters, float* sink, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HSGPT_H */
