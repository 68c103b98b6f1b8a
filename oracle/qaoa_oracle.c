/*
 * Plain FP64 CPU oracle for QAOA statevector simulation.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call this file;
 * only the tests, the smoke check and the benchmark's CPU baseline leg use it. It shares no
 * code, header or table with the GPU library.
 *
 * What it computes (JuliQAOA, Golden et al., SC-W 2023):
 *   - the cost diagonal C(x) over the feasible set S (Sec. 2.1, "Pre-Computation"):
 *     S = all n-bit strings, or the strings of Hamming weight k in increasing integer order;
 *     index x = sum_i x_i 2^i, vertex i <-> bit i. The evolution takes C as a list of FP64
 *     values, one per feasible state (Sec. 3: the objective is handed over as a list of values
 *     over the states); the MaxCut table is one such list, computed exactly in integers;
 *   - the p-round state of Eq. (1): |b,g> = e^{-i b_p H_M} e^{-i g_p H_C} ... e^{-i b_1 H_M}
 *     e^{-i g_1 H_C} |psi0>, phase separator first in every round, with H_C|x> = C(x)|x>;
 *   - H_M = sum_q X_q (transverse field, Sec. 2.1), applied qubit by qubit as the 2x2 rotation
 *     e^{-i b X_q} = cos b I - i sin b X_q (the factorisation behind Eq. (2));
 *   - H_M = |psi0><psi0| (Grover mixer, Sec. 2.4) with psi0 the equal superposition over S:
 *     e^{-i b H_M} = I + (e^{-i b} - 1)|psi0><psi0|, applied as psi += (e^{-i b} - 1) <psi0|psi> psi0;
 *   - H_M = sum_i X_i X_{i+1} + Y_i Y_{i+1} (ring mixer, Sec. 2.1; i + 1 mod n) on weight k:
 *     the same construction with only cyclically adjacent swaps;
 *   - H_M = sum_{i<j} X_i X_j + Y_i Y_j (clique mixer, Sec. 2.1) restricted to weight k: it
 *     maps |x> to 2|y> for every y obtained from x by moving one 1 to a 0 position;
 *     e^{-i b H_M} psi is formed by a scaled Taylor series of the sparse matrix;
 *   - <C> = sum_x |psi(x)|^2 C(x) (the objective of Sec. 1), Neumaier-compensated;
 *   - d<C>/d(beta, gamma) by the adjoint (reverse) recursion: for k = p..1,
 *       g_beta_k  = 2 Im <lambda| H_M |phi>,   (phi, lambda) <- e^{+i b_k H_M} (phi, lambda),
 *       g_gamma_k = 2 Im <lambda| H_C |phi>,   (phi, lambda) <- e^{+i g_k H_C} (phi, lambda),
 *     starting from phi = psi_p and lambda = H_C psi_p. Sec. 2.3 obtains this gradient by
 *     reverse-mode AD; the recursion above is the same reverse sweep written out by hand.
 *   Angles are laid out [beta_1..beta_p, gamma_1..gamma_p] (first code listing, Sec. 3).
 *
 * Everything is FP64 with libm cos/sin; loops are plain and in the paper's order.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ subspace enumeration */

/* Number of k-subsets of n. */
int64_t orc_binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
    return r;
}

static int popcount64(uint64_t x) {
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

/* Feasible set S. k < 0: all 2^n integers 0..2^n-1. k >= 0: the integers with exactly k
 * one-bits in increasing order, found by scanning 0..2^n-1 (plain, not Gosper's walk). */
int64_t orc_states(int n, int k, uint64_t *out) {
    uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    int64_t cnt = 0;
    for (uint64_t x = 0;; x++) {
        if (k < 0 || popcount64(x) == k) {
            if (out) out[cnt] = x;
            cnt++;
        }
        if (x == full) break;
    }
    return cnt;
}

/* ------------------------------------------------------------------ step (a): cost table */

/* MaxCut value of basis string x: sum over edges of w_e [x_u != x_v]. */
static int64_t maxcut_value(uint64_t x, int m, const int32_t *u, const int32_t *v, const int32_t *w) {
    int64_t c = 0;
    for (int e = 0; e < m; e++) {
        uint64_t bu = (x >> u[e]) & 1u, bv = (x >> v[e]) & 1u;
        if (bu != bv) c += (w ? w[e] : 1);
    }
    return c;
}

/* C(x) for every x in S (order of orc_states). Returns |S| or -1 on bad input. */
int64_t orc_cost_table(int n, int m, const int32_t *u, const int32_t *v, const int32_t *w,
                       int k, int64_t *out) {
    if (n < 1 || n > 34) return -1;
    for (int e = 0; e < m; e++)
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n || u[e] == v[e]) return -1;
    if (k < 0) {
        int64_t N = 1ll << n;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; x++) out[x] = maxcut_value((uint64_t)x, m, u, v, w);
        return N;
    }
    int64_t N = orc_binom(n, k);
    uint64_t *st = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    if (!st) return -1;
    orc_states(n, k, st);
    for (int64_t r = 0; r < N; r++) out[r] = maxcut_value(st[r], m, u, v, w);
    free(st);
    return N;
}

/* ------------------------------------------------------------------ compensated sums */

typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_val(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ steps (b) and (c) */

/* psi(x) <- e^{-i gamma C(x)} psi(x). */
void orc_apply_phase(int64_t N, double gamma, const double *cost, cplx *psi) {
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
        double a = -gamma * cost[x];
        psi[x] *= cos(a) + I * sin(a);
    }
}

/* psi <- prod_q e^{-i beta X_q} psi, qubit by qubit: for each pair (x, x + 2^q) with bit q
 * of x clear, (a, b) <- (cos(beta) a - i sin(beta) b, -i sin(beta) a + cos(beta) b). */
void orc_apply_x_mixer(int n, double beta, cplx *psi) {
    double c = cos(beta), s = sin(beta);
    int64_t N = 1ll << n;
    for (int q = 0; q < n; q++) {
        int64_t bit = 1ll << q;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; x++) {
            if (x & bit) continue;
            cplx a = psi[x], b = psi[x | bit];
            psi[x] = c * a - I * s * b;
            psi[x | bit] = -I * s * a + c * b;
        }
    }
}

/* out <- (sum_q X_q) psi, formed directly: out(x) = sum_q psi(x xor 2^q). */
void orc_apply_x_sum(int n, const cplx *psi, cplx *out) {
    int64_t N = 1ll << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
        cplx acc = 0;
        for (int q = 0; q < n; q++) acc += psi[x ^ (1ll << q)];
        out[x] = acc;
    }
}

/* <psi0|psi> for the equal superposition psi0 over N states: sum_x psi(x) / sqrt(N). */
static cplx overlap_uniform(int64_t N, const cplx *psi) {
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;   /* Neumaier on both parts */
    for (int64_t x = 0; x < N; x++) {
        double a = creal(psi[x]), b = cimag(psi[x]);
        double t = sr + a; cr += fabs(sr) >= fabs(a) ? (sr - t) + a : (a - t) + sr; sr = t;
        t = si + b; ci += fabs(si) >= fabs(b) ? (si - t) + b : (b - t) + si; si = t;
    }
    return ((sr + cr) + I * (si + ci)) / sqrt((double)N);
}

/* Grover mixer (Sec. 2.4): psi <- psi + (e^{-i beta} - 1) <psi0|psi> psi0. */
void orc_apply_grover_mixer(int64_t N, double beta, cplx *psi) {
    cplx c = (cexp(-I * beta) - 1.0) * overlap_uniform(N, psi) / sqrt((double)N);
    for (int64_t x = 0; x < N; x++) psi[x] += c;
}

/* H_G psi = psi0 <psi0|psi>: the constant vector <psi0|psi> / sqrt(N). */
static void grover_sum(int64_t N, const cplx *psi, cplx *out) {
    cplx c = overlap_uniform(N, psi) / sqrt((double)N);
    for (int64_t x = 0; x < N; x++) out[x] = c;
}

/* Index of state y in the increasing list st[0..N) (binary search); -1 if absent. */
static int64_t find_state(const uint64_t *st, int64_t N, uint64_t y) {
    int64_t lo = 0, hi = N - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (st[mid] == y) return mid;
        if (st[mid] < y) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Neighbour lists of the clique mixer on weight-k strings: nb[r*deg + j] = index of the
 * state reached from st[r] by moving one 1-bit to a 0-bit (deg = k(n-k)). */
int64_t orc_clique_neighbours(int n, int k, const uint64_t *st, int64_t N, int64_t *nb) {
    int deg = k * (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; r++) {
        uint64_t x = st[r];
        int j = 0;
        for (int a = 0; a < n; a++) {
            if (!((x >> a) & 1u)) continue;
            for (int b = 0; b < n; b++) {
                if ((x >> b) & 1u) continue;
                uint64_t y = (x & ~(1ull << a)) | (1ull << b);
                nb[r * deg + j] = find_state(st, N, y);
                j++;
            }
        }
    }
    return deg;
}

/* Neighbour lists of the ring mixer sum_i X_i X_{i+1} + Y_i Y_{i+1} (i + 1 taken mod n, so the
 * ring closes for n >= 3) on weight-k strings: nb[r*deg + e] = index of the state reached from
 * st[r] by swapping the bits of ring edge e, or -1 when they are equal (deg = ring edges). */
int64_t orc_ring_neighbours(int n, int k, const uint64_t *st, int64_t N, int64_t *nb) {
    (void)k;
    int deg = n >= 3 ? n : (n == 2 ? 1 : 0);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; r++) {
        uint64_t x = st[r];
        for (int e = 0; e < deg; e++) {
            int a = e, b = (e + 1) % n;
            if (((x >> a) & 1u) == ((x >> b) & 1u)) { nb[r * deg + e] = -1; continue; }
            nb[r * deg + e] = find_state(st, N, x ^ (1ull << a) ^ (1ull << b));
        }
    }
    return deg;
}

/* out <- H psi for a swap mixer on the weight-k subspace: every neighbour (nb >= 0)
 * contributes 2. */
static void clique_matvec(int64_t N, int deg, const int64_t *nb, const cplx *psi, cplx *out) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; r++) {
        cplx acc = 0;
        for (int j = 0; j < deg; j++)
            if (nb[r * deg + j] >= 0) acc += 2.0 * psi[nb[r * deg + j]];
        out[r] = acc;
    }
}

/* psi <- e^{-i beta H} psi for a swap mixer given by its neighbour lists (deg per state) by
 * a scaled Taylor series: s steps with |beta| * ||H||_1 / s <= 1 (||H||_1 <= 2 deg), each
 * step summing terms until they fall below 1e-18 relative (at most 60 terms). */
void orc_apply_swap_mixer(int deg, const int64_t *nb, int64_t N, double beta, cplx *psi);

/* psi <- e^{-i beta H_clique} psi (deg = k (n - k) neighbours per state). */
void orc_apply_clique_mixer(int n, int k, const int64_t *nb, int64_t N, double beta, cplx *psi) {
    orc_apply_swap_mixer(k * (n - k), nb, N, beta, psi);
}

void orc_apply_swap_mixer(int deg, const int64_t *nb, int64_t N, double beta, cplx *psi) {
    double norm1 = 2.0 * deg;
    int steps = (int)ceil(fabs(beta) * norm1);
    if (steps < 1) steps = 1;
    double h = beta / steps;
    cplx *term = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *acc = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    for (int st = 0; st < steps; st++) {
        memcpy(term, psi, sizeof(cplx) * (size_t)N);
        memcpy(acc, psi, sizeof(cplx) * (size_t)N);
        double ref = 0;
        for (int64_t r = 0; r < N; r++) ref += cabs(psi[r]);
        for (int j = 1; j <= 60; j++) {
            clique_matvec(N, deg, nb, term, tmp);
            double tn = 0;
            for (int64_t r = 0; r < N; r++) {
                term[r] = (-I * h / j) * tmp[r];
                acc[r] += term[r];
                tn += cabs(term[r]);
            }
            if (tn <= 1e-18 * ref) break;
        }
        memcpy(psi, acc, sizeof(cplx) * (size_t)N);
    }
    free(term); free(tmp); free(acc);
}

/* ------------------------------------------------------------------ step (d): expectation */

/* E = sum |psi|^2 C, Nrm = sum |psi|^2 (Neumaier, sequential). */
double orc_expect(int64_t N, const double *cost, const cplx *psi, double *nrm_out) {
    nsum e = {0, 0}, nr = {0, 0};
    for (int64_t x = 0; x < N; x++) {
        double pr = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
        nsum_add(&e, pr * cost[x]);
        nsum_add(&nr, pr);
    }
    if (nrm_out) *nrm_out = nsum_val(&nr);
    return nsum_val(&e);
}

/* Im sum conj(a) b (Neumaier). */
static double im_inner(int64_t N, const cplx *a, const cplx *b) {
    nsum s = {0, 0};
    for (int64_t x = 0; x < N; x++) nsum_add(&s, cimag(conj(a[x]) * b[x]));
    return nsum_val(&s);
}

/* Im sum conj(a) C b (Neumaier). */
static double im_inner_c(int64_t N, const double *cost, const cplx *a, const cplx *b) {
    nsum s = {0, 0};
    for (int64_t x = 0; x < N; x++) nsum_add(&s, cimag(conj(a[x]) * b[x]) * cost[x]);
    return nsum_val(&s);
}

/* ------------------------------------------------------------------ Eq. (1), both mixers */

typedef struct {
    int n, k;              /* k < 0: all 2^n states; else the weight-k states */
    int grover;            /* 1: Grover mixer on those states; 0: X mixer (k < 0) or a swap
                              mixer (k >= 0: clique, or ring when ring = 1) */
    int ring;
    int64_t N;
    int deg;               /* swap mixer: neighbour slots per state */
    const int64_t *nb;     /* swap mixer neighbour lists (NULL otherwise) */
} mixer_t;

static void apply_mixer(const mixer_t *m, double beta, cplx *psi) {
    if (m->grover) orc_apply_grover_mixer(m->N, beta, psi);
    else if (m->k < 0) orc_apply_x_mixer(m->n, beta, psi);
    else orc_apply_swap_mixer(m->deg, m->nb, m->N, beta, psi);
}

static void apply_mixer_sum(const mixer_t *m, const cplx *psi, cplx *out) {
    if (m->grover) grover_sum(m->N, psi, out);
    else if (m->k < 0) orc_apply_x_sum(m->n, psi, out);
    else clique_matvec(m->N, m->deg, m->nb, psi, out);
}

/* Initial state: psi0 if given, else the uniform superposition over S (Sec. 3: the default
 * start is the equal superposition over all states, or over the weight-k states). */
static void init_state(int64_t N, const cplx *psi0, cplx *psi) {
    if (psi0) { memcpy(psi, psi0, sizeof(cplx) * (size_t)N); return; }
    double a = 1.0 / sqrt((double)N);
    for (int64_t x = 0; x < N; x++) psi[x] = a;
}

static void evolve(const mixer_t *m, int p, const double *angles, const double *cost,
                   const cplx *psi0, cplx *psi) {
    init_state(m->N, psi0, psi);
    for (int r = 0; r < p; r++) {
        orc_apply_phase(m->N, angles[p + r], cost, psi);    /* e^{-i gamma_r H_C} */
        apply_mixer(m, angles[r], psi);                      /* e^{-i beta_r H_M} */
    }
}

/* mixer code: 0 = X (k < 0) or clique (k >= 0); 1 = Grover; 2 = ring (k >= 0) */
static int make_mixer(int n, int k, int code, mixer_t *m, int64_t **nb_store) {
    m->n = n; m->k = k; m->grover = code == 1; m->ring = code == 2; m->nb = NULL; m->deg = 0; *nb_store = NULL;
    if (k < 0) { m->N = 1ll << n; return code == 2 ? -1 : 0; }
    m->N = orc_binom(n, k);
    if (m->grover) return 0;
    uint64_t *st = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m->N);
    int deg = m->ring ? (n >= 3 ? n : (n == 2 ? 1 : 0)) : k * (n - k);
    m->deg = deg;
    int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m->N * (deg > 0 ? deg : 1)));
    if (!st || !nb) { free(st); free(nb); return -1; }
    orc_states(n, k, st);
    if (m->ring) orc_ring_neighbours(n, k, st, m->N, nb);
    else orc_clique_neighbours(n, k, st, m->N, nb);
    free(st);
    m->nb = nb; *nb_store = nb;
    return 0;
}

/* Final state psi_p of Eq. (1). k < 0: X mixer; k >= 0: clique mixer on weight k. */
/* mixer: 0 = X (k < 0) or clique (k >= 0); 1 = Grover on the feasible set; 2 = ring (k >= 0). */
int orc_qaoa_state_m(int n, int k, int mixer, int p, const double *angles, const double *cost,
                     const cplx *psi0, cplx *psi_out) {
    mixer_t m; int64_t *nb;
    if (make_mixer(n, k, mixer, &m, &nb)) return -1;
    evolve(&m, p, angles, cost, psi0, psi_out);
    free(nb);
    return 0;
}

/* <C> (raw E and Nrm) for one angle set. */
int orc_qaoa_expect_m(int n, int k, int mixer, int p, const double *angles, const double *cost,
                      const cplx *psi0, double *E, double *Nrm) {
    mixer_t m; int64_t *nb;
    if (make_mixer(n, k, mixer, &m, &nb)) return -1;
    cplx *psi = (cplx *)malloc(sizeof(cplx) * (size_t)m.N);
    if (!psi) { free(nb); return -1; }
    evolve(&m, p, angles, cost, psi0, psi);
    *E = orc_expect(m.N, cost, psi, Nrm);
    free(psi); free(nb);
    return 0;
}

/* <C> and its gradient [d/dbeta_1..p, d/dgamma_1..p] by the adjoint recursion (header). */
int orc_qaoa_grad_m(int n, int k, int mixer, int p, const double *angles, const double *cost,
                    const cplx *psi0, double *E, double *Nrm, double *grad) {
    mixer_t m; int64_t *nb;
    if (make_mixer(n, k, mixer, &m, &nb)) return -1;
    int64_t N = m.N;
    cplx *phi = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *lam = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!phi || !lam || !tmp) { free(phi); free(lam); free(tmp); free(nb); return -1; }
    evolve(&m, p, angles, cost, psi0, phi);
    *E = orc_expect(N, cost, phi, Nrm);
    for (int64_t x = 0; x < N; x++) lam[x] = cost[x] * phi[x];             /* lambda = H_C psi_p */
    for (int r = p - 1; r >= 0; r--) {
        apply_mixer_sum(&m, phi, tmp);                                     /* H_M phi */
        grad[r] = 2.0 * im_inner(N, lam, tmp);                              /* d/dbeta_r */
        apply_mixer(&m, -angles[r], phi);                                   /* undo mixer */
        apply_mixer(&m, -angles[r], lam);
        grad[p + r] = 2.0 * im_inner_c(N, cost, lam, phi);                  /* d/dgamma_r */
        orc_apply_phase(N, -angles[p + r], cost, phi);                      /* undo phase */
        orc_apply_phase(N, -angles[p + r], cost, lam);
    }
    free(phi); free(lam); free(tmp); free(nb);
    return 0;
}

/* The same with the default mixer of the state space (X for k < 0, clique for k >= 0). */
int orc_qaoa_state(int n, int k, int p, const double *angles, const double *cost, const cplx *psi0,
                   cplx *psi_out) {
    return orc_qaoa_state_m(n, k, 0, p, angles, cost, psi0, psi_out);
}
int orc_qaoa_expect(int n, int k, int p, const double *angles, const double *cost, const cplx *psi0,
                    double *E, double *Nrm) {
    return orc_qaoa_expect_m(n, k, 0, p, angles, cost, psi0, E, Nrm);
}
int orc_qaoa_grad(int n, int k, int p, const double *angles, const double *cost, const cplx *psi0,
                  double *E, double *Nrm, double *grad) {
    return orc_qaoa_grad_m(n, k, 0, p, angles, cost, psi0, E, Nrm, grad);
}

/* Thread count OpenMP would use (for reporting the CPU baseline). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
#else
int orc_num_threads(void) { return 1; }
#endif

/* C(x) at the given basis strings only (sampled checks of very large tables). */
int orc_cost_values(int n, int m, const int32_t *u, const int32_t *v, const int32_t *w,
                    const uint64_t *xs, int64_t count, int64_t *out) {
    if (n < 1 || n > 63) return -1;
    for (int e = 0; e < m; e++)
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n || u[e] == v[e]) return -1;
    for (int64_t i = 0; i < count; i++) out[i] = maxcut_value(xs[i], m, u, v, w);
    return 0;
}
