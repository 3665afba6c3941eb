/*
 * hsgref.c -- plain FP64 CPU oracle for the parallel-tempering hot path of the
 * three-dimensional Heisenberg spin glass (Hasenbusch & Schaefer,
 * arXiv:1006.4247).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the product path never does.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * Every routine is the plain definition, or the algorithm's steps in the order
 * the method gives them, written for clarity, not speed.  Loops run over sites
 * in ascending natural order; the only parallelism is an OpenMP loop over
 * independent replicas (each replica has its own random stream, so results do
 * not depend on the thread count).
 *
 * Sources:
 *   model and Hamiltonian        -- paper Sec. I, Eq. (2)
 *   local field S_x              -- paper Sec. III.A, Eq. (bigS)
 *   W/B checkerboard split       -- paper Sec. III.A
 *   heat-bath / overrelaxation   -- paper Sec. III.C
 *   replica exchange acceptance  -- paper Sec. I, Eq. (1)
 *   overlap, susceptibility, E   -- paper Sec. II, Eq. (eq:over) and following
 *   round trips                  -- paper Sec. IV.B
 *   decimated exchange           -- paper Sec. III.A, Eqs. (xxxY), (HI), (eq:aswap)
 *   cooling / heating exchange   -- paper Sec. III.B
 *   annealed (nonequilibrium) swap -- cited prior art of Sec. I (Opps & Schofield
 *     2001; Ballard & Jarzynski 2009); the protocol below is the standard
 *     nonequilibrium-candidate construction, which reduces to Eq. (1) at K = 0.
 *   Philox4x32-10                -- Salmon, Moraes, Dror & Shaw, SC'11
 *   Box-Muller (cosine branch)   -- Box & Muller 1958
 *   orthonormal frame            -- Duff et al., JCGT 6(1) 2017 ("Building an
 *                                   Orthonormal Basis, Revisited")
 */
#include "hsgref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al. 2011): ten rounds of two 32x32->64 products,  */
/* key bumped by the Weyl constants between rounds.                           */
/* ------------------------------------------------------------------------- */
void hsgref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod0, prod1;
        uint32_t y0, y1, y2, y3;
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        y1 = (uint32_t)prod1;
        y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 23 random bits m: r = (m + 1/2) 2^-23, exactly representable in binary32. */
double hsgref_u01_24(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* 52 random bits m: r = (m + 1/2) 2^-52, exactly representable in binary64. */
double hsgref_u01_52(uint32_t w0, uint32_t w1)
{
    uint64_t m = ((uint64_t)w0 << 20) | (uint64_t)(w1 >> 12);
    return ((double)m + 0.5) * (1.0 / 4503599627370496.0);
}

static void key_of_seed(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t w[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = c0; ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    key_of_seed(seed, key);
    hsgref_philox4x32_10(ctr, key, w);
}

#define TAG_COUPLING 1u
#define TAG_INIT 2u
#define TAG_HEATBATH 3u
#define TAG_SWAP 4u
#define TAG_DECIMATE 5u      /* heat-bath re-insertion after a decimated exchange */
#define TAG_DECIMATE_ROLE 6u /* which sublattice the first pair decimates */

/* ------------------------------------------------------------------------- */
/* Lattice: periodic simple cubic, x = i + L(j + L k); W = even, B = odd.    */
/* ------------------------------------------------------------------------- */
int hsgref_parity(int L, int x)
{
    int i = x % L, j = (x / L) % L, k = x / (L * L);
    return (i + j + k) & 1;
}

int hsgref_compressed_index(int L, int x)
{
    int i = x % L, rest = x / L; /* rest = j + L k */
    return (i / 2) + (L / 2) * rest;
}

int hsgref_neighbor(int L, int x, int dir)
{
    int i = x % L, j = (x / L) % L, k = x / (L * L);
    switch (dir) {
    case 0: i = (i + 1) % L; break;
    case 1: i = (i + L - 1) % L; break;
    case 2: j = (j + 1) % L; break;
    case 3: j = (j + L - 1) % L; break;
    case 4: k = (k + 1) % L; break;
    default: k = (k + L - 1) % L; break;
    }
    return i + L * (j + L * k);
}

/* ------------------------------------------------------------------------- */
/* Initialisation                                                             */
/* ------------------------------------------------------------------------- */

/* Quenched couplings J_xy ~ N(0,1) (paper Sec. I): one Philox block per bond
 * (x, mu) of sample s; Box-Muller, cosine branch, from two 52-bit uniforms. */
void hsgref_init_couplings(int L, int n_samples, uint32_t sample_base, uint64_t seed,
                           int round_f32, double* J)
{
    int N = L * L * L, s, x, mu;
    for (s = 0; s < n_samples; ++s)
        for (x = 0; x < N; ++x)
            for (mu = 0; mu < 3; ++mu) {
                uint32_t w[4];
                double r1, r2, g;
                draw(seed, (uint32_t)x, (uint32_t)mu, sample_base + (uint32_t)s,
                     TAG_COUPLING << 24, w);
                r1 = hsgref_u01_52(w[0], w[1]);
                r2 = hsgref_u01_52(w[2], w[3]);
                g = sqrt(-2.0 * log(r1)) * cos(2.0 * M_PI * r2);
                if (round_f32) g = (double)(float)g;
                J[((size_t)s * N + x) * 3 + mu] = g;
            }
}

/* Random start: uniform on the unit sphere (z uniform in [-1,1], azimuth
 * uniform); cold start: (1,0,0) as in the paper's equilibration study. */
void hsgref_init_spins(int L, int n_slots, uint32_t slot_base, uint64_t seed,
                       int cold, int round_f32, double* s)
{
    int N = L * L * L, n, x, a;
    for (n = 0; n < n_slots; ++n)
        for (x = 0; x < N; ++x) {
            double v[3];
            if (cold) {
                v[0] = 1.0; v[1] = 0.0; v[2] = 0.0;
            } else {
                uint32_t w[4];
                double r1, r2, z, rho, phi;
                draw(seed, (uint32_t)x, 0u, slot_base + (uint32_t)n, TAG_INIT << 24, w);
                r1 = hsgref_u01_52(w[0], w[1]);
                r2 = hsgref_u01_52(w[2], w[3]);
                z = 2.0 * r1 - 1.0;
                rho = 2.0 * sqrt(r1 * (1.0 - r1)); /* sqrt(1 - z^2) */
                phi = 2.0 * M_PI * r2;
                v[0] = rho * cos(phi);
                v[1] = rho * sin(phi);
                v[2] = z;
            }
            for (a = 0; a < 3; ++a) {
                double val = round_f32 ? (double)(float)v[a] : v[a];
                s[((size_t)n * N + x) * 3 + a] = val;
            }
        }
}

/* ------------------------------------------------------------------------- */
/* Local field, Eq. (bigS): S_x = sum over the six neighbours y of J_xy s_y,  */
/* summed in the order +x, -x, +y, -y, +z, -z.  The bond to x - e_mu is the   */
/* forward bond J(x - e_mu, mu) of the neighbour.                             */
/* ------------------------------------------------------------------------- */
void hsgref_local_field(int L, const double* J, const double* s, int x, double S[3])
{
    int mu, a;
    S[0] = S[1] = S[2] = 0.0;
    for (mu = 0; mu < 3; ++mu) {
        int xp = hsgref_neighbor(L, x, 2 * mu);
        int xm = hsgref_neighbor(L, x, 2 * mu + 1);
        double jp = J[(size_t)x * 3 + mu];
        double jm = J[(size_t)xm * 3 + mu];
        for (a = 0; a < 3; ++a) S[a] += jp * s[(size_t)xp * 3 + a];
        for (a = 0; a < 3; ++a) S[a] += jm * s[(size_t)xm * 3 + a];
    }
}

/* ------------------------------------------------------------------------- */
/* Heat-bath update of one spin (paper Sec. III.C).  The component of the new */
/* spin along S_x has density proportional to exp(R c) on [-1,1], R = beta|S|; */
/* the paper inverts its distribution function as c = ln(z + (1/z - z) r)/R   */
/* with z = exp(-R).  The identical expression used here,                     */
/*     w = 1 - c = -log1p((1 - r) expm1(-2R)) / R,                            */
/* stays finite for every R > 0 and keeps full precision as R -> 0.  The two  */
/* orthogonal components are sqrt(1 - c^2) (sin phi, cos phi), phi = 2 pi r2,  */
/* in the frame (e1, e2) of Duff et al. around n = S/|S| (sign +1 iff n_z >= 0).*/
/* If R == 0 (beta = 0 or S = 0) the new spin is uniform: c = 2 r1 - 1.        */
/* ------------------------------------------------------------------------- */
void hsgref_heatbath_spin(const double S[3], double beta, double r1, double r2, double out[3])
{
    double nrm = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    double R = beta * nrm;
    double n[3], w, c, st, sgn, a, b, e1[3], e2[3], phi, sp, cp;
    int k;
    if (nrm > 0.0) {
        n[0] = S[0] / nrm; n[1] = S[1] / nrm; n[2] = S[2] / nrm;
    } else {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    }
    if (R >= 1e-300) {
        w = -log1p((1.0 - r1) * expm1(-2.0 * R)) / R;
    } else {
        w = 2.0 * (1.0 - r1); /* c = 2 r1 - 1 */
    }
    c = 1.0 - w;
    st = sqrt(w * (2.0 - w)); /* sin(theta) = sqrt(1 - c^2) */
    sgn = (n[2] >= 0.0) ? 1.0 : -1.0;
    a = -1.0 / (sgn + n[2]);
    b = n[0] * n[1] * a;
    e1[0] = 1.0 + sgn * n[0] * n[0] * a;
    e1[1] = sgn * b;
    e1[2] = -sgn * n[0];
    e2[0] = b;
    e2[1] = sgn + n[1] * n[1] * a;
    e2[2] = -n[1];
    phi = 2.0 * M_PI * r2;
    sp = sin(phi);
    cp = cos(phi);
    for (k = 0; k < 3; ++k) out[k] = c * n[k] + st * (sp * e1[k] + cp * e2[k]);
}

/* Overrelaxation (paper Sec. III.C): reflect s about S, s' = 2 (s.S)/S^2 S - s.
 * If S = 0 the update is the identity (any energy-preserving involution would
 * do; the paper does not treat this case). */
void hsgref_overrelax_spin(const double s[3], const double S[3], double out[3])
{
    double ss = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    int k;
    if (ss > 0.0) {
        double f = 2.0 * (s[0] * S[0] + s[1] * S[1] + s[2] * S[2]) / ss;
        for (k = 0; k < 3; ++k) out[k] = f * S[k] - s[k];
    } else {
        for (k = 0; k < 3; ++k) out[k] = s[k];
    }
}

/* Uniforms of the heat-bath update of site x in slot g, sweep t, half-sweep
 * label hs (= 2 * heat-bath-sweep index + parity).  h is the site's index in
 * its sublattice.  52-bit mode: one Philox block per site.  24-bit mode: one
 * block per pair of sites (h, h + N/4) of the same sublattice, words 0-1 for
 * the first, 2-3 for the second. */
void hsgref_hb_uniforms(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t t,
                        uint32_t hs, int x, double* r1, double* r2)
{
    int N = L * L * L;
    int h = hsgref_compressed_index(L, x);
    uint32_t w[4];
    uint32_t c3 = (TAG_HEATBATH << 24) | ((hs & 0xFFu) << 16);
    if (!rng32) {
        draw(seed, (uint32_t)h, t, slot_global, c3, w);
        *r1 = hsgref_u01_52(w[0], w[1]);
        *r2 = hsgref_u01_52(w[2], w[3]);
    } else {
        int quarter = N / 4;
        int half = h / quarter;
        draw(seed, (uint32_t)(h % quarter), t, slot_global, c3, w);
        *r1 = hsgref_u01_24(w[2 * half]);
        *r2 = hsgref_u01_24(w[2 * half + 1]);
    }
}

/* Batch forms of the single-site pieces above, for tests that ask how an update
 * responds when its field is moved: plain loops over the same functions, no new
 * arithmetic.  fields: S_out[x] = S_x for the sites of `parity` (zeros elsewhere);
 * uniforms: r1[x], r2[x] of the heat-bath at those sites; the `_many` forms apply
 * one update per row of their [n][3] inputs. */
void hsgref_fields(int L, const double* J, const double* s, int parity, double* S_out)
{
    int N = L * L * L, x;
    for (x = 0; x < N; ++x) {
        double* S = S_out + (size_t)x * 3;
        if (hsgref_parity(L, x) == parity) {
            hsgref_local_field(L, J, s, x, S);
        } else {
            S[0] = S[1] = S[2] = 0.0;
        }
    }
}

void hsgref_hb_uniforms_all(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t t,
                            uint32_t hs, int parity, double* r1, double* r2)
{
    int N = L * L * L, x;
    for (x = 0; x < N; ++x) {
        if (hsgref_parity(L, x) == parity) {
            hsgref_hb_uniforms(L, rng32, seed, slot_global, t, hs, x, r1 + x, r2 + x);
        } else {
            r1[x] = r2[x] = 0.0;
        }
    }
}

void hsgref_heatbath_many(int n, const double* S, const double* beta, const double* r1,
                          const double* r2, double* out)
{
    int i;
    for (i = 0; i < n; ++i)
        hsgref_heatbath_spin(S + (size_t)i * 3, beta[i], r1[i], r2[i], out + (size_t)i * 3);
}

void hsgref_overrelax_many(int n, const double* s, const double* S, double* out)
{
    int i;
    for (i = 0; i < n; ++i)
        hsgref_overrelax_spin(s + (size_t)i * 3, S + (size_t)i * 3, out + (size_t)i * 3);
}

/* ------------------------------------------------------------------------- */
/* Energies                                                                   */
/* ------------------------------------------------------------------------- */

/* Eq. (2): H = - sum over bonds J_xy s_x . s_y, each bond (x, mu) once. */
double hsgref_energy(int L, const double* J, const double* s)
{
    int N = L * L * L, x, mu;
    double H = 0.0;
    for (x = 0; x < N; ++x)
        for (mu = 0; mu < 3; ++mu) {
            int y = hsgref_neighbor(L, x, 2 * mu);
            const double* sx = s + (size_t)x * 3;
            const double* sy = s + (size_t)y * 3;
            H -= J[(size_t)x * 3 + mu] * (sx[0] * sy[0] + sx[1] * sy[1] + sx[2] * sy[2]);
        }
    return H;
}

/* -sum_{x in sublattice p} s_x . S_x; every bond has exactly one end in p. */
double hsgref_sublattice_energy(int L, const double* J, const double* s, int parity)
{
    int N = L * L * L, x;
    double H = 0.0;
    for (x = 0; x < N; ++x) {
        double S[3];
        const double* sx = s + (size_t)x * 3;
        if (hsgref_parity(L, x) != parity) continue;
        hsgref_local_field(L, J, s, x, S);
        H -= sx[0] * S[0] + sx[1] * S[1] + sx[2] * S[2];
    }
    return H;
}

/* ------------------------------------------------------------------------- */
/* Half-sweep: update every site of one sublattice (kind 0 = heat-bath,      */
/* 1 = overrelaxation).  Sites of one sublattice do not interact (paper Sec.  */
/* III.A), so the result does not depend on the visiting order; `order`       */
/* (N/2 site indices of that sublattice) may be given to check that.          */
/* ------------------------------------------------------------------------- */
static void update_site(int L, const double* J, double* s, int x, int kind, double beta,
                        uint64_t seed, uint32_t slot_global, uint32_t t, uint32_t hs, int rng32)
{
    double S[3], out[3];
    double* sx = s + (size_t)x * 3;
    hsgref_local_field(L, J, s, x, S);
    if (kind == 0) {
        double r1, r2;
        hsgref_hb_uniforms(L, rng32, seed, slot_global, t, hs, x, &r1, &r2);
        hsgref_heatbath_spin(S, beta, r1, r2, out);
    } else {
        hsgref_overrelax_spin(sx, S, out);
    }
    sx[0] = out[0]; sx[1] = out[1]; sx[2] = out[2];
}

void hsgref_halfsweep(int L, const double* J, double* s, int parity, int kind, double beta,
                      uint64_t seed, uint32_t slot_global, uint32_t t, uint32_t hs, int rng32,
                      const int32_t* order)
{
    int N = L * L * L, x, n;
    if (order) {
        for (n = 0; n < N / 2; ++n)
            update_site(L, J, s, order[n], kind, beta, seed, slot_global, t, hs, rng32);
        return;
    }
    for (x = 0; x < N; ++x)
        if (hsgref_parity(L, x) == parity)
            update_site(L, J, s, x, kind, beta, seed, slot_global, t, hs, rng32);
}

/* One sweep: n_hb heat-bath lattice sweeps then n_or overrelaxation lattice
 * sweeps, each as W then B (forward order).  The adjoint order runs the same
 * half-sweeps in reverse.  A heat-bath half-sweep keeps its label
 * hs = 2*ihb + parity in either order. */
void hsgref_sweep(int L, const double* J, double* s, int n_hb, int n_or, int adjoint,
                  double beta, uint64_t seed, uint32_t slot_global, uint32_t t, int rng32)
{
    int ihb, ior;
    if (!adjoint) {
        for (ihb = 0; ihb < n_hb; ++ihb) {
            hsgref_halfsweep(L, J, s, 0, 0, beta, seed, slot_global, t, (uint32_t)(2 * ihb), rng32, 0);
            hsgref_halfsweep(L, J, s, 1, 0, beta, seed, slot_global, t, (uint32_t)(2 * ihb + 1), rng32, 0);
        }
        for (ior = 0; ior < n_or; ++ior) {
            hsgref_halfsweep(L, J, s, 0, 1, beta, seed, slot_global, t, 0u, rng32, 0);
            hsgref_halfsweep(L, J, s, 1, 1, beta, seed, slot_global, t, 0u, rng32, 0);
        }
    } else {
        for (ior = 0; ior < n_or; ++ior) {
            hsgref_halfsweep(L, J, s, 1, 1, beta, seed, slot_global, t, 0u, rng32, 0);
            hsgref_halfsweep(L, J, s, 0, 1, beta, seed, slot_global, t, 0u, rng32, 0);
        }
        for (ihb = n_hb - 1; ihb >= 0; --ihb) {
            hsgref_halfsweep(L, J, s, 1, 0, beta, seed, slot_global, t, (uint32_t)(2 * ihb + 1), rng32, 0);
            hsgref_halfsweep(L, J, s, 0, 0, beta, seed, slot_global, t, (uint32_t)(2 * ihb), rng32, 0);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Ensembles: S samples x C chains x R slots.  Slot (s,c,r) holds a physical  */
/* configuration; temp_of_slot / slot_of_temp are the temperature labels.    */
/* Global stream indices: slot_global = slot_base + (s C + c) R + r,          */
/* chain_global = chain_base + s C + c.                                       */
/* ------------------------------------------------------------------------- */
void hsgref_sweep_batch(int L, int S, int C, int R, const double* J, double* spins,
                        const double* betas, const int32_t* temp_of_slot, uint32_t* sweep_ctr,
                        uint32_t slot_base, uint64_t seed, int n_sweeps, int n_hb, int n_or,
                        int rng32, double* energy)
{
    int N = L * L * L;
    int n_slot = S * C * R, q;
#pragma omp parallel for schedule(dynamic, 1)
    for (q = 0; q < n_slot; ++q) {
        int smp = q / (C * R), n;
        const double* Js = J + (size_t)smp * N * 3;
        double* sp = spins + (size_t)q * N * 3;
        double beta = betas[temp_of_slot[q]];
        for (n = 0; n < n_sweeps; ++n)
            hsgref_sweep(L, Js, sp, n_hb, n_or, 0, beta, seed, slot_base + (uint32_t)q,
                         sweep_ctr[q] + (uint32_t)n, rng32);
        sweep_ctr[q] += (uint32_t)n_sweeps;
        if (energy) energy[q] = hsgref_energy(L, Js, sp);
    }
}

/* Round trips (paper Sec. IV.B): a configuration completes a trip when it is
 * back at the highest temperature (label 0, smallest beta) after having
 * visited the lowest (label R-1) since its previous visit to label 0.
 * state: 0 = label 0 not yet visited, 1 = heading to R-1, 2 = heading back. */
void hsgref_roundtrip_update(int R, const int32_t* temp_of_slot, int32_t* rt_state,
                             int64_t* rt_trips)
{
    int r;
    for (r = 0; r < R; ++r) {
        int T = temp_of_slot[r];
        if (T == 0) {
            if (rt_state[r] == 2) rt_trips[r] += 1;
            rt_state[r] = 1;
        } else if (T == R - 1) {
            if (rt_state[r] == 1) rt_state[r] = 2;
        }
    }
}

static int pair_selected(int i, int pairing)
{
    if (pairing == 0) return 1;
    if (pairing == 1) return (i % 2) == 0;
    return (i % 2) == 1;
}

static void relabel(int32_t* temp_of_slot, int32_t* slot_of_temp, int i)
{
    int x = slot_of_temp[i], y = slot_of_temp[i + 1];
    slot_of_temp[i] = y;
    slot_of_temp[i + 1] = x;
    temp_of_slot[x] = i + 1;
    temp_of_slot[y] = i;
}

/* Replica exchange, Eq. (1): the configurations at beta_i and beta_{i+1}
 * exchange temperatures with probability
 * min[1, exp((beta_{i+1} - beta_i)(H_{i+1} - H_i))], decided as
 * ln u < (beta_{i+1} - beta_i)(H_{i+1} - H_i).  pairing 0 visits all pairs in
 * ascending order, 1 the even pairs, 2 the odd pairs. */
void hsgref_swap_batch(int S, int C, int R, const double* betas, const double* energy,
                       int32_t* temp_of_slot, int32_t* slot_of_temp, uint32_t* swap_ctr,
                       int64_t* stats, int32_t* rt_state, int64_t* rt_trips,
                       uint32_t chain_base, uint64_t seed, int pairing)
{
    int ch, n_chain = S * C;
    for (ch = 0; ch < n_chain; ++ch) {
        int32_t* tos = temp_of_slot + (size_t)ch * R;
        int32_t* sot = slot_of_temp + (size_t)ch * R;
        const double* en = energy + (size_t)ch * R;
        int64_t* st = stats + (size_t)ch * (R - 1) * 2;
        uint32_t cg = chain_base + (uint32_t)ch;
        uint32_t n = swap_ctr[ch];
        int i;
        for (i = 0; i < R - 1; ++i) {
            uint32_t w[4];
            double u, delta;
            int x, y;
            if (!pair_selected(i, pairing)) continue;
            x = sot[i];
            y = sot[i + 1];
            delta = (betas[i + 1] - betas[i]) * (en[y] - en[x]);
            draw(seed, (uint32_t)i, n, cg, TAG_SWAP << 24, w);
            u = hsgref_u01_52(w[0], w[1]);
            st[2 * i] += 1;
            if (log(u) < delta) {
                relabel(tos, sot, i);
                st[2 * i + 1] += 1;
            }
        }
        swap_ctr[ch] = n + 1;
        hsgref_roundtrip_update(R, tos, rt_state + (size_t)ch * R, rt_trips + (size_t)ch * R);
    }
}

/* ------------------------------------------------------------------------- */
/* Annealed swap (nonequilibrium candidate).  For the pair (a = beta_i,      */
/* b = beta_{i+1}) and a protocol a = l_0 < l_1 < ... < l_K < l_{K+1} = b:     */
/*   up-leg of x (at a):   W_up = sum_{k=0..K} (l_{k+1} - l_k) H(x_k),         */
/*                         x_{k+1} = forward sweep at l_{k+1} of x_k (k < K);  */
/*   down-leg of y (at b): m_k = l_{K+1-k}, W_dn = sum_k (m_{k+1} - m_k) H(y_k),*/
/*                         y_{k+1} = adjoint sweep at m_{k+1} of y_k;          */
/*   accept with min[1, exp(-(W_up + W_dn))], decided as ln u < -(W_up+W_dn). */
/* Accepted: x_K takes temperature b, y_K temperature a.  Rejected: x and y   */
/* keep their states from before the legs.  At K = 0 this is Eq. (1).          */
/* Default protocol (lambda == NULL): l_k = a + k (b - a)/(K + 1).            */
/* ------------------------------------------------------------------------- */
static double anneal_leg(int L, const double* J, double* s, int K, const double* lam_up,
                         int down, int n_hb, int n_or, uint64_t seed, uint32_t slot_global,
                         uint32_t t0, int rng32)
{
    /* lam_up[0..K+1] ascending; the down-leg walks it backwards. */
    double W = 0.0, H = hsgref_energy(L, J, s);
    int k;
    for (k = 0; k <= K; ++k) {
        double cur = down ? lam_up[K + 1 - k] : lam_up[k];
        double nxt = down ? lam_up[K - k] : lam_up[k + 1];
        W += (nxt - cur) * H;
        if (k < K) {
            hsgref_sweep(L, J, s, n_hb, n_or, down, nxt, seed, slot_global, t0 + (uint32_t)k, rng32);
            H = hsgref_energy(L, J, s);
        }
    }
    return W;
}

void hsgref_anneal_batch(int L, int S, int C, int R, const double* J, double* spins,
                         const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                         uint32_t* sweep_ctr, uint32_t* swap_ctr, double* energy,
                         int64_t* stats, int32_t* rt_state, int64_t* rt_trips,
                         uint32_t slot_base, uint32_t chain_base, uint64_t seed, int parity,
                         const int32_t* K, const double* lambda, int K_max, int n_hb, int n_or,
                         int rng32, double* work_out)
{
    int N = L * L * L;
    int n_chain = S * C;
    int n_task = n_chain * (R - 1), task;
    size_t rep = (size_t)N * 3;
    double* wbuf = (double*)calloc((size_t)n_task * 2, sizeof(double));
    double* cand = (double*)malloc((size_t)n_task * 2 * rep * sizeof(double));

    /* legs: every selected pair is independent */
#pragma omp parallel for schedule(dynamic, 1)
    for (task = 0; task < n_task; ++task) {
        int ch = task / (R - 1), i = task % (R - 1), smp = ch / C, k;
        const double* Js = J + (size_t)smp * rep;
        const int32_t* sot = slot_of_temp + (size_t)ch * R;
        int x, y, Ki;
        double* lam;
        if ((i % 2) != parity) continue;
        x = ch * R + sot[i];
        y = ch * R + sot[i + 1];
        Ki = K[i];
        lam = (double*)malloc((size_t)(Ki + 2) * sizeof(double));
        lam[0] = betas[i];
        lam[Ki + 1] = betas[i + 1];
        for (k = 1; k <= Ki; ++k)
            lam[k] = lambda ? lambda[(size_t)i * K_max + (k - 1)]
                            : betas[i] + (double)k * (betas[i + 1] - betas[i]) / (double)(Ki + 1);
        memcpy(cand + (size_t)task * 2 * rep, spins + (size_t)x * rep, rep * sizeof(double));
        memcpy(cand + ((size_t)task * 2 + 1) * rep, spins + (size_t)y * rep, rep * sizeof(double));
        wbuf[2 * task] = anneal_leg(L, Js, cand + (size_t)task * 2 * rep, Ki, lam, 0, n_hb, n_or,
                                    seed, slot_base + (uint32_t)x, sweep_ctr[x], rng32);
        wbuf[2 * task + 1] = anneal_leg(L, Js, cand + ((size_t)task * 2 + 1) * rep, Ki, lam, 1,
                                        n_hb, n_or, seed, slot_base + (uint32_t)y, sweep_ctr[y], rng32);
        free(lam);
    }

    /* decisions, in pair order per chain */
    for (task = 0; task < n_task; ++task) {
        int ch = task / (R - 1), i = task % (R - 1), smp = ch / C;
        int32_t* tos = temp_of_slot + (size_t)ch * R;
        int32_t* sot = slot_of_temp + (size_t)ch * R;
        int64_t* st = stats + (size_t)ch * (R - 1) * 2;
        const double* Js = J + (size_t)smp * rep;
        uint32_t w[4];
        double u, Wsum;
        int x, y;
        if ((i % 2) != parity) {
            if (work_out) { work_out[2 * task] = 0.0; work_out[2 * task + 1] = 0.0; }
            continue;
        }
        x = ch * R + sot[i];
        y = ch * R + sot[i + 1];
        sweep_ctr[x] += (uint32_t)K[i];
        sweep_ctr[y] += (uint32_t)K[i];
        Wsum = wbuf[2 * task] + wbuf[2 * task + 1];
        if (work_out) { work_out[2 * task] = wbuf[2 * task]; work_out[2 * task + 1] = wbuf[2 * task + 1]; }
        draw(seed, (uint32_t)i, swap_ctr[ch], chain_base + (uint32_t)ch, TAG_SWAP << 24, w);
        u = hsgref_u01_52(w[0], w[1]);
        st[2 * i] += 1;
        if (log(u) < -Wsum) {
            memcpy(spins + (size_t)x * rep, cand + (size_t)task * 2 * rep, rep * sizeof(double));
            memcpy(spins + (size_t)y * rep, cand + ((size_t)task * 2 + 1) * rep, rep * sizeof(double));
            energy[x] = hsgref_energy(L, Js, spins + (size_t)x * rep);
            energy[y] = hsgref_energy(L, Js, spins + (size_t)y * rep);
            relabel(tos, sot, i);
            st[2 * i + 1] += 1;
        }
    }
    {
        int ch;
        for (ch = 0; ch < n_chain; ++ch) {
            swap_ctr[ch] += 1;
            hsgref_roundtrip_update(R, temp_of_slot + (size_t)ch * R, rt_state + (size_t)ch * R,
                                    rt_trips + (size_t)ch * R);
        }
    }
    free(cand);
    free(wbuf);
}

/* ------------------------------------------------------------------------- */
/* Decimated exchange (paper Sec. III.A).  The sites of one sublattice D do   */
/* not interact, so integrating their spins out of exp(-beta H) leaves, per   */
/* site z in D, I(beta S_z) = int ds exp(beta s.S_z) = 4 pi sinh(R)/R with    */
/* R = beta |S_z| (Eq. (HI); the measure ds on the unit sphere has total      */
/* 4 pi), S_z the local field of the kept sublattice.  Exchanging the kept    */
/* fields of x (at beta_1) and y (at beta_2) is accepted with Eq. (eq:aswap): */
/*   ln A = sum_{z in D} [h(b2 a_z) - h(b1 a_z) + h(b1 c_z) - h(b2 c_z)],      */
/* a_z = |S_z(x)|, c_z = |S_z(y)|, h(u) = ln(sinh(u)/u) = ln I / (4 pi); the   */
/* constants 4 pi and the 1/R factors cancel between the four terms.          */
/* If accepted, the D spins of both configurations are drawn anew by heat-    */
/* bath at their new temperatures (x at beta_2, y at beta_1); if rejected,    */
/* nothing changes.  The first pair decimates a random sublattice and the     */
/* role alternates from one pair to the next: D_i = (d_0 + i) mod 2.          */
/* ------------------------------------------------------------------------- */

/* h(u) = ln(sinh(u)/u) for u >= 0, written as u + ln((1 - e^{-2u})/(2u)):     */
/* finite for every u, h(0) = 0.                                               */
double hsgref_log_sinhc(double u)
{
    if (u <= 0.0) return 0.0;
    return u + log(-expm1(-2.0 * u) / (2.0 * u));
}

/* ln A of Eq. (eq:aswap) for x at b1 and y at b2, decimating parity d. */
double hsgref_decimated_log_ratio(int L, const double* J, const double* sx, const double* sy,
                                  int d, double b1, double b2)
{
    int N = L * L * L, z;
    double lnA = 0.0;
    for (z = 0; z < N; ++z) {
        double Sa[3], Sc[3], a, c;
        if (hsgref_parity(L, z) != d) continue;
        hsgref_local_field(L, J, sx, z, Sa);
        hsgref_local_field(L, J, sy, z, Sc);
        a = sqrt(Sa[0] * Sa[0] + Sa[1] * Sa[1] + Sa[2] * Sa[2]);
        c = sqrt(Sc[0] * Sc[0] + Sc[1] * Sc[1] + Sc[2] * Sc[2]);
        lnA += hsgref_log_sinhc(b2 * a) - hsgref_log_sinhc(b1 * a)
             + hsgref_log_sinhc(b1 * c) - hsgref_log_sinhc(b2 * c);
    }
    return lnA;
}

/* Uniforms of the re-insertion of site x after pair i of call n: the layout  */
/* of hsgref_hb_uniforms with counter word 1 = n and word 3 = tag, pair.      */
void hsgref_decimate_uniforms(int L, int rng32, uint64_t seed, uint32_t slot_global, uint32_t n,
                              uint32_t pair, int x, double* r1, double* r2)
{
    int N = L * L * L;
    int h = hsgref_compressed_index(L, x);
    uint32_t w[4];
    uint32_t c3 = (TAG_DECIMATE << 24) | (pair & 0xFFFFu);
    if (!rng32) {
        draw(seed, (uint32_t)h, n, slot_global, c3, w);
        *r1 = hsgref_u01_52(w[0], w[1]);
        *r2 = hsgref_u01_52(w[2], w[3]);
    } else {
        int quarter = N / 4;
        int half = h / quarter;
        draw(seed, (uint32_t)(h % quarter), n, slot_global, c3, w);
        *r1 = hsgref_u01_24(w[2 * half]);
        *r2 = hsgref_u01_24(w[2 * half + 1]);
    }
}

/* Heat-bath draw of every site of parity d at beta (fields from the other    */
/* sublattice, which stays fixed).                                            */
static void reinsert(int L, const double* J, double* s, int d, double beta, uint64_t seed,
                     uint32_t slot_global, uint32_t n, uint32_t pair, int rng32)
{
    int N = L * L * L, z;
    for (z = 0; z < N; ++z) {
        double S[3], r1, r2;
        if (hsgref_parity(L, z) != d) continue;
        hsgref_local_field(L, J, s, z, S);
        hsgref_decimate_uniforms(L, rng32, seed, slot_global, n, pair, z, &r1, &r2);
        hsgref_heatbath_spin(S, beta, r1, r2, s + (size_t)z * 3);
    }
}

int hsgref_decimate_role(uint64_t seed, uint32_t chain_global, uint32_t n)
{
    uint32_t w[4];
    draw(seed, 0u, n, chain_global, TAG_DECIMATE_ROLE << 24, w);
    return (int)(w[0] & 1u);
}

void hsgref_decimate_batch(int L, int S, int C, int R, const double* J, double* spins,
                           const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                           uint32_t* swap_ctr, double* energy, int64_t* stats, int32_t* rt_state,
                           int64_t* rt_trips, uint32_t slot_base, uint32_t chain_base,
                           uint64_t seed, int pairing, int rng32, double* log_ratio_out,
                           int32_t* role_out)
{
    int N = L * L * L;
    int ch, n_chain = S * C;
    size_t rep = (size_t)N * 3;
    for (ch = 0; ch < n_chain; ++ch) {
        int smp = ch / C, i;
        const double* Js = J + (size_t)smp * rep;
        int32_t* tos = temp_of_slot + (size_t)ch * R;
        int32_t* sot = slot_of_temp + (size_t)ch * R;
        int64_t* st = stats + (size_t)ch * (R - 1) * 2;
        uint32_t cg = chain_base + (uint32_t)ch;
        uint32_t n = swap_ctr[ch];
        int d0 = hsgref_decimate_role(seed, cg, n);
        for (i = 0; i < R - 1; ++i) {
            uint32_t w[4];
            double u, lnA;
            int x, y, d;
            size_t gx, gy;
            if (log_ratio_out) log_ratio_out[(size_t)ch * (R - 1) + i] = 0.0;
            if (role_out) role_out[(size_t)ch * (R - 1) + i] = -1;
            if (!pair_selected(i, pairing)) continue;
            d = (d0 + i) & 1;
            x = sot[i];
            y = sot[i + 1];
            gx = (size_t)ch * R + (size_t)x;
            gy = (size_t)ch * R + (size_t)y;
            lnA = hsgref_decimated_log_ratio(L, Js, spins + gx * rep, spins + gy * rep, d,
                                             betas[i], betas[i + 1]);
            if (log_ratio_out) log_ratio_out[(size_t)ch * (R - 1) + i] = lnA;
            if (role_out) role_out[(size_t)ch * (R - 1) + i] = d;
            draw(seed, (uint32_t)i, n, cg, TAG_SWAP << 24, w);
            u = hsgref_u01_52(w[0], w[1]);
            st[2 * i] += 1;
            if (log(u) < lnA) {
                reinsert(L, Js, spins + gx * rep, d, betas[i + 1], seed, slot_base + (uint32_t)gx,
                         n, (uint32_t)i, rng32);
                reinsert(L, Js, spins + gy * rep, d, betas[i], seed, slot_base + (uint32_t)gy,
                         n, (uint32_t)i, rng32);
                energy[gx] = hsgref_energy(L, Js, spins + gx * rep);
                energy[gy] = hsgref_energy(L, Js, spins + gy * rep);
                relabel(tos, sot, i);
                st[2 * i + 1] += 1;
            }
        }
        swap_ctr[ch] = n + 1;
        hsgref_roundtrip_update(R, tos, rt_state + (size_t)ch * R, rt_trips + (size_t)ch * R);
    }
}

/* ------------------------------------------------------------------------- */
/* Cooling / heating exchange (paper Sec. III.B).  One spin s with field S    */
/* (|S| > 0, n = S/|S|, cos(theta) = s.n, k = eps |S|): cooling turns s       */
/* towards S by alpha = eps |p| = k sin(theta), p = S - (S.s) s, in the plane */
/* of s and S:  s' = s cos(alpha) + (p/|p|) sin(alpha), theta' = theta-alpha.  */
/* For k < 1, theta -> theta' is increasing on [0, pi], so the map is a       */
/* bijection of the sphere; its Jacobian (area ratio) is                      */
/*   |1 - eps S.s| (cos(alpha) - cot(theta) sin(alpha))                       */
/*   = (1 - k cos(theta)) (cos(alpha) - cos(theta) k sinc(alpha)),            */
/* sinc(a) = sin(a)/a, finite at the poles.  Heating is the inverse: theta    */
/* from theta' by Newton's method on theta - k sin(theta) = theta'.           */
/* A lattice cooling C cools every parity-0 spin (fields from parity 1), then */
/* every parity-1 spin (fields from the cooled parity 0); the Jacobian of C is */
/* the product of the site factors.  Heating C^-1 undoes the parity-1 step,   */
/* then the parity-0 step.                                                    */
/* Exchange of x at b1 = beta_i and y at b2 = beta_{i+1}: the proposal       */
/* (x, y) -> (C^-1 y at b1, C x at b2) is an involution, accepted with        */
/*   ln A = b1 H(x) + b2 H(y) - b1 H(C^-1 y) - b2 H(C x)                     */
/*          + ln det J_C(x) - ln det J_C(C^-1 y),                            */
/* decided as ln u < ln A; eps = 0 is Eq. (1).  If k >= 1 at a site of either */
/* map the pair is rejected (the map is then not a bijection).               */
/* ------------------------------------------------------------------------- */

static double sinc(double a)
{
    if (fabs(a) < 1e-4) return 1.0 - a * a / 6.0;
    return sin(a) / a;
}

/* log of the Jacobian of the cooling map at a spin with cos(theta) = c,
 * sin(theta) = st, k = eps |S|. */
static double cool_log_jacobian(double c, double st, double k)
{
    double alpha = k * st;
    return log(1.0 - k * c) + log(cos(alpha) - c * k * sinc(alpha));
}

/* Cool one spin; returns the log Jacobian, or NAN if eps |S| >= 1. */
double hsgref_cool_spin(const double s[3], const double S[3], double eps, double out[3])
{
    double nS = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    double k = eps * nS, Ss, c, p[3], np, st, alpha, ca, sa;
    int a;
    if (k >= 1.0) return NAN;
    if (nS == 0.0) {
        for (a = 0; a < 3; ++a) out[a] = s[a];
        return 0.0;
    }
    Ss = S[0] * s[0] + S[1] * s[1] + S[2] * s[2];
    c = Ss / nS;
    for (a = 0; a < 3; ++a) p[a] = S[a] - Ss * s[a];
    np = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    st = np / nS;
    alpha = eps * np;
    ca = cos(alpha);
    sa = sin(alpha);
    for (a = 0; a < 3; ++a) out[a] = (np > 0.0) ? s[a] * ca + p[a] / np * sa : s[a];
    return cool_log_jacobian(c, st, k);
}

/* Heat one spin (the inverse of cooling); returns the log Jacobian of the
 * cooling map at the result, or NAN if eps |S| >= 1. */
double hsgref_heat_spin(const double sp[3], const double S[3], double eps, double out[3])
{
    double nS = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    double k = eps * nS, Ss, q[3], nq, thp, th, alpha, ca, sa;
    int a, it;
    if (k >= 1.0) return NAN;
    if (nS == 0.0) {
        for (a = 0; a < 3; ++a) out[a] = sp[a];
        return 0.0;
    }
    Ss = S[0] * sp[0] + S[1] * sp[1] + S[2] * sp[2];
    for (a = 0; a < 3; ++a) q[a] = S[a] - Ss * sp[a];
    nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    thp = atan2(nq, Ss); /* theta' in [0, pi] */
    th = thp + k * sin(thp);
    for (it = 0; it < 50; ++it) {
        double g = th - k * sin(th) - thp;
        double d = g / (1.0 - k * cos(th));
        th -= d;
        if (fabs(d) <= 1e-16 * (1.0 + th)) break;
    }
    alpha = th - thp;
    ca = cos(alpha);
    sa = sin(alpha);
    for (a = 0; a < 3; ++a) out[a] = (nq > 0.0) ? sp[a] * ca - q[a] / nq * sa : sp[a];
    return cool_log_jacobian(cos(th), sin(th), k);
}

/* Lattice cooling (heat = 0) or heating (heat = 1) in place; returns the log
 * Jacobian of the cooling map (at s before cooling, or at the heated result). */
double hsgref_coolheat(int L, const double* J, double* s, double eps, int heat)
{
    int N = L * L * L, step, z;
    double logdet = 0.0;
    for (step = 0; step < 2; ++step) {
        int par = heat ? 1 - step : step;
        for (z = 0; z < N; ++z) {
            double S[3], o[3], ld;
            if (hsgref_parity(L, z) != par) continue;
            hsgref_local_field(L, J, s, z, S);
            ld = heat ? hsgref_heat_spin(s + (size_t)z * 3, S, eps, o)
                      : hsgref_cool_spin(s + (size_t)z * 3, S, eps, o);
            s[(size_t)z * 3 + 0] = o[0];
            s[(size_t)z * 3 + 1] = o[1];
            s[(size_t)z * 3 + 2] = o[2];
            logdet += ld;
        }
    }
    return logdet;
}

void hsgref_coolheat_batch(int L, int S, int C, int R, const double* J, double* spins,
                           const double* betas, int32_t* temp_of_slot, int32_t* slot_of_temp,
                           uint32_t* swap_ctr, double* energy, int64_t* stats, int32_t* rt_state,
                           int64_t* rt_trips, uint32_t chain_base, uint64_t seed, int pairing,
                           double eps, double* log_ratio_out, double* logdet_out,
                           const double* eps_pair)
{
    int N = L * L * L;
    int ch, n_chain = S * C;
    size_t rep = (size_t)N * 3;
    double* cx = (double*)malloc(rep * sizeof(double));
    double* cy = (double*)malloc(rep * sizeof(double));
    for (ch = 0; ch < n_chain; ++ch) {
        int smp = ch / C, i;
        const double* Js = J + (size_t)smp * rep;
        int32_t* tos = temp_of_slot + (size_t)ch * R;
        int32_t* sot = slot_of_temp + (size_t)ch * R;
        int64_t* st = stats + (size_t)ch * (R - 1) * 2;
        uint32_t cg = chain_base + (uint32_t)ch;
        uint32_t n = swap_ctr[ch];
        for (i = 0; i < R - 1; ++i) {
            uint32_t w[4];
            double u, lnA, ldx, ldy, hx, hy, b1 = betas[i], b2 = betas[i + 1];
            size_t gx, gy;
            size_t o = (size_t)ch * (R - 1) + i;
            if (log_ratio_out) log_ratio_out[o] = 0.0;
            if (logdet_out) { logdet_out[2 * o] = 0.0; logdet_out[2 * o + 1] = 0.0; }
            if (!pair_selected(i, pairing)) continue;
            gx = (size_t)ch * R + (size_t)sot[i];
            gy = (size_t)ch * R + (size_t)sot[i + 1];
            memcpy(cx, spins + gx * rep, rep * sizeof(double));
            memcpy(cy, spins + gy * rep, rep * sizeof(double));
            /* the map's parameter: one for every pair, or pair i's own (Sec. IV suggests
             * tuning it for each pair of temperatures) */
            {
                double e_i = eps_pair ? eps_pair[i] : eps;
                ldx = hsgref_coolheat(L, Js, cx, e_i, 0);
                ldy = hsgref_coolheat(L, Js, cy, e_i, 1);
            }
            hx = hsgref_energy(L, Js, cx);
            hy = hsgref_energy(L, Js, cy);
            lnA = b1 * energy[gx] + b2 * energy[gy] - b1 * hy - b2 * hx + ldx - ldy;
            if (log_ratio_out) log_ratio_out[o] = lnA;
            if (logdet_out) { logdet_out[2 * o] = ldx; logdet_out[2 * o + 1] = ldy; }
            draw(seed, (uint32_t)i, n, cg, TAG_SWAP << 24, w);
            u = hsgref_u01_52(w[0], w[1]);
            st[2 * i] += 1;
            if (log(u) < lnA) { /* false for NaN: a map that is not a bijection rejects */
                memcpy(spins + gx * rep, cx, rep * sizeof(double));
                memcpy(spins + gy * rep, cy, rep * sizeof(double));
                energy[gx] = hx;
                energy[gy] = hy;
                relabel(tos, sot, i);
                st[2 * i + 1] += 1;
            }
        }
        swap_ctr[ch] = n + 1;
        hsgref_roundtrip_update(R, tos, rt_state + (size_t)ch * R, rt_trips + (size_t)ch * R);
    }
    free(cx);
    free(cy);
}

/* ------------------------------------------------------------------------- */
/* Measurement (paper Sec. II): overlap q_{ab,x} = s^(1)_{a,x} s^(2)_{b,x}    */
/* between the chain-0 and chain-1 configurations at the same temperature,    */
/* Q_ab = sum_x q_{ab,x}, chi = (1/N) sum_ab Q_ab^2; energy per site e = H/N   */
/* (the paper's E is -e).  Outputs are indexed by temperature.                */
/* ------------------------------------------------------------------------- */
void hsgref_measure_batch(int L, int S, int C, int R, const double* spins, const double* energy,
                          const int32_t* slot_of_temp, double* Q, double* chi, double* e)
{
    int N = L * L * L, smp, b, c;
    size_t rep = (size_t)N * 3;
    for (smp = 0; smp < S; ++smp) {
        for (c = 0; c < C; ++c)
            for (b = 0; b < R; ++b) {
                int q = (smp * C + c) * R + slot_of_temp[(size_t)(smp * C + c) * R + b];
                if (e) e[(size_t)(smp * C + c) * R + b] = energy[q] / (double)N;
            }
        if (C < 2) continue;
        for (b = 0; b < R; ++b) {
            int q1 = (smp * C + 0) * R + slot_of_temp[(size_t)(smp * C + 0) * R + b];
            int q2 = (smp * C + 1) * R + slot_of_temp[(size_t)(smp * C + 1) * R + b];
            const double* s1 = spins + (size_t)q1 * rep;
            const double* s2 = spins + (size_t)q2 * rep;
            double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, sum = 0.0;
            int x, al, be;
            for (x = 0; x < N; ++x)
                for (al = 0; al < 3; ++al)
                    for (be = 0; be < 3; ++be)
                        M[al * 3 + be] += s1[(size_t)x * 3 + al] * s2[(size_t)x * 3 + be];
            for (al = 0; al < 9; ++al) sum += M[al] * M[al];
            if (Q)
                for (al = 0; al < 9; ++al) Q[((size_t)smp * R + b) * 9 + al] = M[al];
            if (chi) chi[(size_t)smp * R + b] = sum / (double)N;
        }
    }
}

int hsgref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (n >= 1); the timing of a reference run
 * on one thread uses it. */
void hsgref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
