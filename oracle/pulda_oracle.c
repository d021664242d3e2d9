/*
 * pulda_oracle.c -- plain, slow, single-threaded CPU oracle for the Polya-urn
 * partially collapsed LDA sampler (Terenin, Magnusson, Jonsson, Draper,
 * "Polya Urn Latent Dirichlet Allocation: a doubly sparse massively parallel
 * sampler", arXiv 1704.03581).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or constant generator with the GPU library: every table it
 * uses it builds itself, from the definitions below.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so pulda_oracle.c -lm
 * (-ffp-contract=off: every fp64 expression is evaluated exactly as written.)
 *
 * Layouts (oracle-internal, chosen for readability): counts n and the Phi
 * draws are topic-major K x V arrays, n[k*V + v], as in Table 1 (n : K x V).
 * Documents are CSR: doc_off[D+1], words[N]; topic indicators z[N] (uint16).
 *
 * What it computes, in the paper's order (Algorithm 2, Section 3):
 *   1. Phi-step: for every topic row k, phi_k ~ PPU(n_k + beta) (Definition of
 *      the Poisson Polya urn, Section 3.3; parameters of eq. for LDA):
 *      gamma_kv ~ Pois(beta + n_kv), phi_kv = gamma_kv / sum_v gamma_kv.
 *      Pois(beta + l) for 1 <= l <= L by a Walker alias table, l > L by a
 *      rounded Gaussian draw (Section 3.4).  Cells with n_kv = 0 draw
 *      Pois(beta); they are found by geometric jumps over each column (see
 *      or_phi_counts).
 *   2. z-step: for every document, for every token i in stored order,
 *      P(z_i = k) propto phi_{k,v(i)} alpha_k + phi_{k,v(i)} m^{-i}_{d,k}
 *      (Algorithm 2, Section 3.5): u ~ U(0,1), u_sigma = u (sigma_a + sigma_b);
 *      if u_sigma < sigma_a draw from the per-word alias table of the a-part,
 *      else walk the b-part.  The oracle walks the b-part densely over all k
 *      (zeros add exactly 0.0), which is the plain definition the sparse walk
 *      must reproduce.
 *   3. Count rebuild n, m from z (Table 1: statistics of the current iteration).
 *   4. Collapsed log joint log p(w | z, beta) + log p(z | alpha) (the
 *      "marginal unnormalized log-posterior for z" of Section 4).
 *   5. Fold-in of a new document against a fixed Phi (z-step restricted to
 *      that document, Phi held fixed).
 *   6. The Phi-step of Algorithm 1 (the partially collapsed sampler the
 *      urn replaces): phi_k ~ Dir(n_k + beta) through Gamma draws (see
 *      or_phi_dirichlet); its z-step is step 2 on the resulting Phi.
 *   7. The held-out log-likelihood of a new document by the left-to-right
 *      algorithm, which Section 4 uses to compare the two samplers' topics
 *      (see or_heldout_ltr).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by the sampler seed, with the
 * counter naming what is drawn (see the TAG_* constants).  The GPU library
 * implements the same published generator independently.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* entries of a zero-truncated Poisson threshold table (rates up to 16 saturate
 * well before) */
#define ZTP_CAP 64

enum { TAG_INIT = 0, TAG_PHI_CELL = 1, TAG_PHI_PRIOR = 2, TAG_Z = 3, TAG_FOLDIN_INIT = 4, TAG_FOLDIN_Z = 5,
       TAG_PHI_GAMMA = 6, TAG_LTR = 7 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 S-box, the key  */
/* bumped by the Weyl constants between rounds.                              */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t tag, uint32_t r[4])
{
    uint32_t ctr[4] = {a, b, c, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, r);
}

/* uniform integer in [0, n) from one 32-bit word: floor(r * n / 2^32) */
static uint32_t mulhi(uint32_t r, uint32_t n) { return (uint32_t)(((uint64_t)r * n) >> 32); }
/* 24-bit uniform in [0, 1): exactly representable in fp32 and fp64 */
static double u24(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }
/* 53-bit uniform in [0, 1) from two words */
static double u53(uint32_t ra, uint32_t rb)
{
    return ((double)(ra >> 5) * 67108864.0 + (double)(rb >> 6)) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Walker alias table (Walker 1977), built by Vose's method (Vose 1991) with  */
/* FIFO work lists in ascending index order.  p_j = (w_j * n) / W with W the  */
/* ascending sum of the weights.  Entries never paired keep probability 1:    */
/* threshold 2^32-1 and alias = self, so that the draw                       */
/*   j = mulhi(r_a, n);  x = (r_b < thr[j]) ? j : alias[j]                    */
/* returns j whatever r_b is.                                                */
/* ------------------------------------------------------------------------ */
void or_vose(const double *w, int32_t n, uint32_t *thr, int32_t *alias)
{
    double W = 0.0;
    for (int32_t j = 0; j < n; j++) W += w[j];
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t *small = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n + 1));
    int32_t *large = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    double *prob = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t s_head = 0, s_tail = 0, l_head = 0, l_tail = 0;
    for (int32_t j = 0; j < n; j++) {
        p[j] = (w[j] * (double)n) / W;
        alias[j] = j;
        prob[j] = 1.0;
        if (p[j] < 1.0) small[s_tail++] = j; else large[l_tail++] = j;
    }
    while (s_head < s_tail && l_head < l_tail) {
        int32_t s = small[s_head++];
        int32_t g = large[l_head];
        prob[s] = p[s];
        alias[s] = g;
        p[g] = (p[g] + p[s]) - 1.0;
        if (p[g] < 1.0) { l_head++; small[s_tail++] = g; }
    }
    for (int32_t j = 0; j < n; j++) {
        if (prob[j] >= 1.0) { thr[j] = 0xFFFFFFFFu; alias[j] = j; }
        else thr[j] = (uint32_t)floor(prob[j] * 4294967296.0);
    }
    free(p); free(small); free(large); free(prob);
}

/* ------------------------------------------------------------------------ */
/* Poisson(beta + l) alias tables for l = 1..L (Section 3.4).                 */
/* Support x = 0..X_l with X_l = ceil(lam + 10 sqrt(lam) + 10); the mass      */
/* beyond X_l is below 1e-20 for every l <= 100.                             */
/* pmf(x) = exp(x ln lam - lam - lgamma(x + 1)), normalised by its ascending  */
/* sum inside Vose's construction.                                           */
/* ------------------------------------------------------------------------ */
int32_t or_pois_support(double beta, int32_t l)
{
    double lam = beta + (double)l;
    return (int32_t)ceil(lam + 10.0 * sqrt(lam) + 10.0) + 1;   /* number of entries */
}

void or_pois_table(double beta, int32_t l, uint32_t *thr, int32_t *alias)
{
    double lam = beta + (double)l;
    int32_t n = or_pois_support(beta, l);
    double *pmf = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t x = 0; x < n; x++)
        pmf[x] = exp((double)x * log(lam) - lam - lgamma((double)x + 1.0));
    or_vose(pmf, n, thr, alias);
    free(pmf);
}

/* Zero-truncated Pois(beta) by inverse CDF over x = 1..6:
 * T_x = floor(2^32 P(X <= x | X >= 1)), value = 1 + #{x in 1..5 : r >= T_x}. */
int32_t or_ztp_thresholds(double beta, uint32_t *T, int32_t cap)
{
    double norm = -expm1(-beta);            /* P(X >= 1) */
    double cdf = 0.0, term = exp(-beta);    /* term = P(X = x) */
    int32_t n = 0;
    for (int x = 1; x <= cap; x++) {
        term = term * beta / (double)x;
        cdf += term;
        double c = cdf / norm;
        double t = floor(c * 4294967296.0);
        T[n++] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
        /* at least 5 entries; then stop at the first that saturates: the
         * mass above it is below the 2^-32 resolution of r2 */
        if (x >= 5 && T[n - 1] == 0xFFFFFFFFu) break;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Initial state: z_i uniform on {0..K-1}.                                    */
/* ------------------------------------------------------------------------ */
void or_init_z(int64_t N, int32_t K, uint64_t seed, uint16_t *z)
{
    for (int64_t i = 0; i < N; i++) {
        uint32_t r[4];
        draw4(seed, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0, TAG_INIT, r);
        z[i] = (uint16_t)mulhi(r[0], (uint32_t)K);
    }
}

/* ------------------------------------------------------------------------ */
/* Count rebuild (Table 1): n_kv = #{i : w_i = v, z_i = k},                   */
/* m_dk = #{i in d : z_i = k}, n_k = sum_v n_kv.  n is K x V, m is D x K      */
/* (m may be NULL).                                                          */
/* ------------------------------------------------------------------------ */
void or_counts(int64_t D, int32_t K, int32_t V, const int64_t *doc_off, const int32_t *words,
               const uint16_t *z, int32_t *n, int64_t *nk, int32_t *m)
{
    memset(n, 0, sizeof(int32_t) * (size_t)K * (size_t)V);
    memset(nk, 0, sizeof(int64_t) * (size_t)K);
    if (m) memset(m, 0, sizeof(int32_t) * (size_t)D * (size_t)K);
    for (int64_t d = 0; d < D; d++)
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            n[(size_t)z[i] * V + words[i]] += 1;
            nk[z[i]] += 1;
            if (m) m[(size_t)d * K + z[i]] += 1;
        }
}

/* ------------------------------------------------------------------------ */
/* Phi-step, part 1: the Poisson draws gamma_kv (the unnormalised PPU row).   */
/*   counted cell n_kv = l >= 1: ctr (v, k, t, PHI_CELL) -> r0..r3;           */
/*     l <= L: x = Pois alias table of l at (r0, r1);                          */
/*     l >  L: rounded Gaussian N(lam, lam), lam = beta + l:                  */
/*       g = sqrt(-2 ln(1 - u53(r0,r1))) cos(2 pi u53(r2,r3)),                 */
/*       x = max(0, floor(lam + sqrt(lam) g + 0.5)).                           */
/*   cells with n_kv = 0 draw Pois(beta): each is nonzero independently with  */
/*     probability q = 1 - exp(-beta), so the nonzero cells of a column are   */
/*     found by geometric jumps: with ctr (v, j, t, PHI_PRIOR), j = 0, 1, ...:  */
/*       e = -ln(1 - u53(r0,r1)) / beta  (P(gap >= g) = (1-q)^g = exp(-beta g)),*/
/*       pos <- pos + 1 + floor(e) starting from pos = -1, stop once pos >= K; */
/*     a marked cell with n_kv = 0 gets a zero-truncated Pois(beta) value from */
/*     r2; marks that land on counted cells are ignored (they carry their own */
/*     draw).  This is the same law as one Pois(beta) draw per zero cell.     */
/* ------------------------------------------------------------------------ */
void or_phi_counts(int32_t K, int32_t V, double beta, const double *beta_v, int32_t L, uint64_t seed, uint32_t t,
                   const int32_t *n, int32_t *gam)
{
    /* beta_v (V priors, or NULL for the symmetric beta): with a vector,
     * Pois(beta_v + l) of a counted cell is the sum of Pois(l) (alias tables
     * of integer rates, a rounded Gaussian of rate l above L) and the cell's
     * Pois(beta_v) prior mark, which the column's jumps draw for every cell,
     * counted or not: the same law, with the per-word rate kept in the one
     * place it varies */
    const double tb = beta_v ? 0.0 : beta;     /* the tables' rate offset */
    /* Poisson tables, rebuilt here every call: plain, not fast */
    int32_t *sizes = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L + 1));
    uint32_t **thr = (uint32_t **)malloc(sizeof(uint32_t *) * (size_t)(L + 1));
    int32_t **ali = (int32_t **)malloc(sizeof(int32_t *) * (size_t)(L + 1));
    for (int32_t l = 1; l <= L; l++) {
        sizes[l] = or_pois_support(tb, l);
        thr[l] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)sizes[l]);
        ali[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)sizes[l]);
        or_pois_table(tb, l, thr[l], ali[l]);
    }
    uint32_t T[ZTP_CAP];
    int32_t nT = or_ztp_thresholds(beta, T, ZTP_CAP);
    const double two_pi = 6.283185307179586476925286766559;

    for (int32_t v = 0; v < V; v++) {
        const double bv = beta_v ? beta_v[v] : beta;
        if (beta_v) nT = or_ztp_thresholds(bv, T, ZTP_CAP);
        for (int32_t k = 0; k < K; k++) {
            int32_t l = n[(size_t)k * V + v];
            int32_t x = 0;
            if (l >= 1) {
                uint32_t r[4];
                draw4(seed, (uint32_t)v, (uint32_t)k, t, TAG_PHI_CELL, r);
                if (l <= L) {
                    uint32_t j = mulhi(r[0], (uint32_t)sizes[l]);
                    x = (r[1] < thr[l][j]) ? (int32_t)j : ali[l][j];
                } else {
                    double lam = tb + (double)l;
                    double g = sqrt(-2.0 * log(1.0 - u53(r[0], r[1]))) * cos(two_pi * u53(r[2], r[3]));
                    double y = floor(lam + sqrt(lam) * g + 0.5);
                    x = y > 0.0 ? (int32_t)y : 0;
                }
            }
            gam[(size_t)k * V + v] = x;
        }
        /* prior marks over zero-count cells of column v */
        int64_t pos = -1;
        for (uint32_t j = 0;; j++) {
            uint32_t r[4];
            draw4(seed, (uint32_t)v, j, t, TAG_PHI_PRIOR, r);
            double e = -log(1.0 - u53(r[0], r[1])) / bv;
            int64_t gap = (int64_t)floor(e);
            if (pos + 1 + gap >= (int64_t)K) break;
            pos = pos + 1 + gap;
            int32_t x = 1;
            for (int q = 0; q < nT; q++) if (r[2] >= T[q]) x++;
            if (n[(size_t)pos * V + v] == 0) gam[(size_t)pos * V + v] = x;
            else if (beta_v) gam[(size_t)pos * V + v] += x;
        }
    }
    for (int32_t l = 1; l <= L; l++) { free(thr[l]); free(ali[l]); }
    free(sizes); free(thr); free(ali);
}

/* ------------------------------------------------------------------------ */
/* Phi-step, part 2: normalise each row (Definition of the PPU):              */
/*   S_k = sum_v gamma_kv (exact integer), phi_kv = fp32(gamma_kv / S_k)       */
/*   (quotient in fp64, rounded once to fp32).  A row with S_k = 0 is left    */
/*   empty (the PPU is defined only for a nonzero sum).                       */
/* ------------------------------------------------------------------------ */
int32_t or_phi_normalise(int32_t K, int32_t V, const int32_t *gam, int64_t *S, float *phi)
{
    int32_t empty_rows = 0;
    for (int32_t k = 0; k < K; k++) {
        int64_t s = 0;
        for (int32_t v = 0; v < V; v++) s += gam[(size_t)k * V + v];
        S[k] = s;
        if (s == 0) empty_rows++;
        for (int32_t v = 0; v < V; v++) {
            int32_t g = gam[(size_t)k * V + v];
            phi[(size_t)k * V + v] = g > 0 ? (float)((double)g / (double)s) : 0.0f;
        }
    }
    return empty_rows;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 Phi-step: phi_k ~ Dir(n_k + beta) for every topic row k, by    */
/* the Gamma representation of the Dirichlet (Section 3.3):                   */
/*   gamma_kv ~ G(beta + n_kv, 1),  phi_kv = gamma_kv / sum_v gamma_kv.        */
/* Gamma draws by Marsaglia and Tsang (2000), the method Section 3.4 names.   */
/* For shape a >= 1, with d = a - 1/3 and c = 1 / sqrt(9 d):                   */
/*   x ~ N(0, 1), t = 1 + c x; reject if t <= 0; v = t^3, u ~ U(0, 1);         */
/*   accept d v if u < 1 - 0.0331 x^4 (their squeeze) or                       */
/*   log u < x^2 / 2 + d (1 - v + log v); else try again.                       */
/* For a < 1 their boost: G(a) = G(a + 1) * U^(1/a), U^(1/a) taken as          */
/* exp(log(U) / a).                                                           */
/* Random numbers: attempt j of cell (k, v) at sweep t uses Philox counter     */
/* (v, k, t, PHI_GAMMA + 256 j):                                              */
/*   x = sqrt(-2 log u(r0)) cos(2 pi u(r1))   (Box and Muller 1958),           */
/*   u = u(r2), and r3 of attempt 0 is the boost's U,                          */
/* with u(r) = (r + 1/2) / 2^32 in (0, 1).  After GAMMA_TRIES rejected          */
/* attempts (probability below 0.05^(2^20)) the draw is d.                    */
/* ------------------------------------------------------------------------ */
#define GAMMA_TRIES (1u << 20)

static double u32o(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

double or_gamma_draw(double a, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double a1 = a < 1.0 ? a + 1.0 : a;
    const double d = a1 - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double g = d;
    uint32_t boost = 0;
    for (uint32_t j = 0; j < GAMMA_TRIES; j++) {
        uint32_t r[4];
        draw4(seed, c0, c1, c2, TAG_PHI_GAMMA + (j << 8), r);
        if (j == 0) boost = r[3];
        double x = sqrt(-2.0 * log(u32o(r[0]))) * cos(two_pi * u32o(r[1]));
        double t1 = 1.0 + c * x;
        if (t1 <= 0.0) continue;
        double v = t1 * t1 * t1;
        double u = u32o(r[2]);
        double x2 = x * x;
        if (u < 1.0 - 0.0331 * (x2 * x2) || log(u) < 0.5 * x2 + d * (1.0 - v + log(v))) {
            g = d * v;
            break;
        }
    }
    if (a < 1.0) g = g * exp(log(u32o(boost)) / a);
    return g;
}

/* Rows: S_k = sum_v gamma_kv, ascending v, in fp64; phi_kv = fp32(gamma_kv / */
/* S_k) (quotient in fp64, rounded once).  A cell whose phi is below the      */
/* smallest normal fp32 (2^-126: zero or subnormal) is set to zero, so the    */
/* sparse Phi is the set of cells with a normal fp32 value.  A row with       */
/* S_k = 0 is empty.  gam, phi: topic-major K x V.  Returns the empty rows.   */
int32_t or_phi_dirichlet(int32_t K, int32_t V, double beta, const double *beta_v, uint64_t seed, uint32_t t,
                         const int32_t *n, double *gam, double *S, float *phi)
{
    const float flt_min = 1.17549435082228750797e-38f;
    int32_t empty_rows = 0;
    for (int32_t k = 0; k < K; k++)
        for (int32_t v = 0; v < V; v++)
            gam[(size_t)k * V + v] = or_gamma_draw((beta_v ? beta_v[v] : beta) + (double)n[(size_t)k * V + v], seed,
                                                   (uint32_t)v, (uint32_t)k, t);
    for (int32_t k = 0; k < K; k++) {
        double s = 0.0;
        for (int32_t v = 0; v < V; v++) s += gam[(size_t)k * V + v];
        S[k] = s;
        if (s == 0.0) empty_rows++;
        for (int32_t v = 0; v < V; v++) {
            float f = s > 0.0 ? (float)(gam[(size_t)k * V + v] / s) : 0.0f;
            phi[(size_t)k * V + v] = f >= flt_min ? f : 0.0f;
        }
    }
    return empty_rows;
}

/* ------------------------------------------------------------------------ */
/* Phi-step, part 3: per-word tables for the a-part (Section 3.5).             */
/* For column v, its nonzero entries in ascending topic order e = 0..n_v-1     */
/* have weights w_e = alpha_k * phi_kv (fp64).  sigma_a[v] = ascending sum;    */
/* the alias table over the entries is Vose's (or_vose).  Output arrays are   */
/* CSC by word: colptr[V+1] (int64), topic[nnz], thr[nnz], alias_topic[nnz]   */
/* (the topic the alias slot points to).  Returns nnz.  With colptr == NULL   */
/* only counts.                                                               */
/* ------------------------------------------------------------------------ */
int64_t or_word_tables(int32_t K, int32_t V, const double *alpha, const float *phi,
                       int64_t *colptr, uint16_t *topic, float *phival, uint32_t *thr,
                       uint16_t *alias_topic, double *sigma_a)
{
    int64_t nnz = 0;
    double *w = (double *)malloc(sizeof(double) * (size_t)K);
    int32_t *ks = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    uint32_t *th = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K);
    int32_t *al = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    for (int32_t v = 0; v < V; v++) {
        int32_t nv = 0;
        for (int32_t k = 0; k < K; k++) {
            float f = phi[(size_t)k * V + v];
            if (f > 0.0f) { ks[nv] = k; w[nv] = alpha[k] * (double)f; nv++; }
        }
        if (colptr) {
            colptr[v] = nnz;
            double s = 0.0;
            for (int32_t e = 0; e < nv; e++) s += w[e];
            sigma_a[v] = s;
            if (nv > 0) or_vose(w, nv, th, al);
            for (int32_t e = 0; e < nv; e++) {
                topic[nnz + e] = (uint16_t)ks[e];
                phival[nnz + e] = phi[(size_t)ks[e] * V + v];
                thr[nnz + e] = th[e];
                alias_topic[nnz + e] = (uint16_t)ks[al[e]];
            }
        }
        nnz += nv;
    }
    if (colptr) colptr[V] = nnz;
    free(w); free(ks); free(th); free(al);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* One token draw (Section 3.5).                                              */
/*   Z = sigma_a + sigma_b, sigma_b = sum_k phi_kv m_k (ascending fp64 sum;   */
/*   each product is exact in fp64);  x = u24(r0) Z.                          */
/*   x < sigma_a:  a-part, alias slot j = mulhi(r1, n_v), keep j if           */
/*                 r2 < thr[j], else its alias.                               */
/*   otherwise:    b-part, y = x - sigma_a, the smallest k whose running sum  */
/*                 of b_k = phi_kv m_k exceeds y (if rounding leaves none, the*/
/*                 largest k with b_k > 0).                                   */
/* Returns the topic; *branch_a = 1 for the a-part.  Also returns, through    */
/* the optional out-parameters, x, Z and the running sum at the chosen topic  */
/* (for the tie classification of the replay check).                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t K, V;
    const float *phi;          /* K x V */
    const int64_t *colptr;     /* word tables, CSC */
    const uint16_t *topic;
    const uint32_t *thr;
    const uint16_t *alias_topic;
    const double *sigma_a;
} or_model;

static int32_t draw_token(const or_model *M, int32_t v, const int32_t *m, const uint32_t r[4],
                          int *branch_a, double *x_out, double *Z_out)
{
    const int32_t K = M->K, V = M->V;
    double sb = 0.0;
    for (int32_t k = 0; k < K; k++) sb += (double)M->phi[(size_t)k * V + v] * (double)m[k];
    double sa = M->sigma_a[v];
    double Z = sa + sb;
    double x = u24(r[0]) * Z;
    if (x_out) *x_out = x;
    if (Z_out) *Z_out = Z;
    if (x < sa) {
        int64_t c0 = M->colptr[v];
        uint32_t nv = (uint32_t)(M->colptr[v + 1] - c0);
        uint32_t j = mulhi(r[1], nv);
        *branch_a = 1;
        return (r[2] < M->thr[c0 + j]) ? M->topic[c0 + j] : M->alias_topic[c0 + j];
    }
    *branch_a = 0;
    double y = x - sa, c = 0.0;
    int32_t last = -1;
    for (int32_t k = 0; k < K; k++) {
        double b = (double)M->phi[(size_t)k * V + v] * (double)m[k];
        if (b > 0.0) {
            c += b;
            last = k;
            if (c > y) return k;
        }
    }
    return last;
}

/* ------------------------------------------------------------------------ */
/* z-step over all documents (sequential Gibbs within each document, tokens   */
/* in stored order; documents are independent given Phi).  A token whose      */
/* word has an empty Phi column has a conditional 0/0: it keeps its topic and */
/* is counted as degenerate.  Returns the number of degenerate tokens; the    */
/* optional stats get sum of J_i = min(K_d^{-i}, K_v) and the a-branch count. */
/* ------------------------------------------------------------------------ */
int64_t or_z_step(int64_t D, int32_t K, int32_t V, const int64_t *doc_off, const int32_t *words,
                  uint16_t *z, uint64_t seed, uint32_t t, const float *phi, const int64_t *colptr,
                  const uint16_t *topic, const uint32_t *thr, const uint16_t *alias_topic,
                  const double *sigma_a, int64_t *stats /* [sum_J, sum_A] or NULL */)
{
    or_model M = {K, V, phi, colptr, topic, thr, alias_topic, sigma_a};
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int64_t degenerate = 0, sumJ = 0, sumA = 0;
    for (int64_t d = 0; d < D; d++) {
        memset(m, 0, sizeof(int32_t) * (size_t)K);
        int32_t kd = 0;
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            if (m[z[i]]++ == 0) kd++;
        }
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            int32_t v = words[i];
            int32_t kold = z[i];
            if (--m[kold] == 0) kd--;
            uint32_t r[4];
            draw4(seed, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), t, TAG_Z, r);
            int64_t nv = colptr[v + 1] - colptr[v];
            if (nv == 0) {
                if (m[kold]++ == 0) kd++;
                degenerate++;
                continue;
            }
            sumJ += (kd < nv) ? kd : nv;
            int a;
            int32_t knew = draw_token(&M, v, m, r, &a, NULL, NULL);
            sumA += a;
            if (m[knew]++ == 0) kd++;
            z[i] = (uint16_t)knew;
        }
    }
    free(m);
    if (stats) { stats[0] = sumJ; stats[1] = sumA; }
    return degenerate;
}

/* ------------------------------------------------------------------------ */
/* The same z-step, doubly sparse (Section 3.5, cost in Section 3.6): the     */
/* b-terms phi_kv m_k are nonzero only where both the document's counts and   */
/* the word's Phi column are, so each token iterates the smaller of the two:  */
/* the document's topics with a nonzero count (kept as an ascending list      */
/* beside the dense m) or the word's column (its CSC entries, ascending).     */
/* Either way the nonzero products are added in ascending topic order, the    */
/* order of the dense sum above, whose zero terms add exactly 0.0; so z, the  */
/* statistics and the random numbers used are bit-identical to or_z_step.     */
/* This is the mode the CPU throughput baseline times.                        */
/* ------------------------------------------------------------------------ */
int64_t or_z_step_sparse(int64_t D, int32_t K, int32_t V, const int64_t *doc_off, const int32_t *words,
                         uint16_t *z, uint64_t seed, uint32_t t, const float *phi, const int64_t *colptr,
                         const uint16_t *topic, const uint32_t *thr, const uint16_t *alias_topic,
                         const double *sigma_a, int64_t *stats /* [sum_J, sum_A] or NULL */)
{
    int32_t *m = (int32_t *)calloc((size_t)K, sizeof(int32_t));
    int32_t *lst = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);   /* nonzero topics, ascending */
    int32_t *bk = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);    /* topics of the iterated side */
    double *bv = (double *)malloc(sizeof(double) * (size_t)K);       /* their b-terms */
    int64_t degenerate = 0, sumJ = 0, sumA = 0;
    for (int64_t d = 0; d < D; d++) {
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) m[z[i]]++;
        int32_t kd = 0;
        for (int32_t k = 0; k < K; k++)
            if (m[k]) lst[kd++] = k;
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            int32_t v = words[i];
            int32_t kold = z[i];
            if (--m[kold] == 0) {
                /* kold leaves the list */
                int32_t j = 0;
                while (lst[j] != kold) j++;
                for (; j + 1 < kd; j++) lst[j] = lst[j + 1];
                kd--;
            }
            uint32_t r[4];
            draw4(seed, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), t, TAG_Z, r);
            int64_t c0 = colptr[v], nv = colptr[v + 1] - c0;
            int32_t knew;
            if (nv == 0) {
                degenerate++;
                knew = kold;
            } else {
                sumJ += (kd < nv) ? kd : nv;
                /* the nonzero b-terms in ascending topic order */
                int32_t nb = 0;
                if (kd <= nv) {
                    for (int32_t j = 0; j < kd; j++) {
                        double b = (double)phi[(size_t)lst[j] * V + v] * (double)m[lst[j]];
                        if (b > 0.0) { bk[nb] = lst[j]; bv[nb] = b; nb++; }
                    }
                } else {
                    for (int64_t e = c0; e < c0 + nv; e++) {
                        int32_t k = topic[e];
                        double b = (double)phi[(size_t)k * V + v] * (double)m[k];
                        if (b > 0.0) { bk[nb] = k; bv[nb] = b; nb++; }
                    }
                }
                double sb = 0.0;
                for (int32_t j = 0; j < nb; j++) sb += bv[j];
                double sa = sigma_a[v];
                double x = u24(r[0]) * (sa + sb);
                if (x < sa) {
                    uint32_t j = mulhi(r[1], (uint32_t)nv);
                    knew = (r[2] < thr[c0 + j]) ? topic[c0 + j] : alias_topic[c0 + j];
                    sumA++;
                } else {
                    double y = x - sa, c = 0.0;
                    knew = -1;
                    for (int32_t j = 0; j < nb && knew < 0; j++) {
                        c += bv[j];
                        if (c > y) knew = bk[j];
                    }
                    if (knew < 0) knew = bk[nb - 1];
                }
            }
            if (m[knew]++ == 0) {
                /* knew enters the list */
                int32_t j = kd;
                while (j > 0 && lst[j - 1] > knew) { lst[j] = lst[j - 1]; j--; }
                lst[j] = knew;
                kd++;
            }
            z[i] = (uint16_t)knew;
        }
        for (int32_t j = 0; j < kd; j++) m[lst[j]] = 0;
    }
    free(m); free(lst); free(bk); free(bv);
    if (stats) { stats[0] = sumJ; stats[1] = sumA; }
    return degenerate;
}

/* ------------------------------------------------------------------------ */
/* Teacher-forced replay of one z-step.  z_before is the state the other      */
/* implementation started from, z_after its result.  Each token is redrawn by */
/* the oracle given the other side's preceding draws in the same document,    */
/* then the other side's draw is taken, so every disagreement is isolated.    */
/* A disagreement is a tie when x lies within tol * Z of the set of x values  */
/* that would have produced the other side's topic (its a-part slot with the  */
/* same r1, r2, or its b-part interval).  out[0] = agreements, out[1] = ties, */
/* out[2] = other disagreements, out[3] = degenerate tokens; worst[0] =       */
/* largest relative distance seen among disagreements (infinite when a value */
/* is not a topic: z_after >= K counts as a disagreement, z_before >= K makes */
/* every token of its document one).  With docs != NULL only the listed      */
/* documents are checked (each is independent given Phi).                     */
/* ------------------------------------------------------------------------ */
void or_replay(int64_t D, int32_t K, int32_t V, const int64_t *doc_off, const int32_t *words,
               const uint16_t *z_before, const uint16_t *z_after, uint64_t seed, uint32_t t,
               const float *phi, const int64_t *colptr, const uint16_t *topic, const uint32_t *thr,
               const uint16_t *alias_topic, const double *sigma_a, double tol, int64_t out[4],
               double worst[1], int64_t *first_bad /* token index or -1 */,
               const int64_t *docs, int64_t n_docs /* documents to check; docs == NULL: all D */)
{
    or_model M = {K, V, phi, colptr, topic, thr, alias_topic, sigma_a};
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    out[0] = out[1] = out[2] = out[3] = 0;
    worst[0] = 0.0;
    *first_bad = -1;
    int64_t nd = docs ? n_docs : D;
    for (int64_t di = 0; di < nd; di++) {
        int64_t d = docs ? docs[di] : di;
        memset(m, 0, sizeof(int32_t) * (size_t)K);
        int64_t bad_start = -1;
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            if (z_before[i] >= K) { bad_start = i; break; }
            m[z_before[i]]++;
        }
        if (bad_start >= 0) {
            /* the starting state holds a value that is not a topic: nothing
             * of this document can be replayed */
            out[2] += doc_off[d + 1] - doc_off[d];
            if (*first_bad < 0) *first_bad = bad_start;
            worst[0] = INFINITY;
            continue;
        }
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) {
            int32_t v = words[i];
            int32_t kold = z_before[i];
            int32_t kg = z_after[i];
            m[kold]--;
            uint32_t r[4];
            draw4(seed, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), t, TAG_Z, r);
            if (colptr[v + 1] == colptr[v]) {
                out[3]++;
                if (kg == kold) out[0]++;
                else { out[2]++; if (*first_bad < 0) *first_bad = i; }
                m[kold]++;   /* the token keeps its topic (0/0 conditional) */
                continue;
            }
            int a;
            double x, Z;
            int32_t ko = draw_token(&M, v, m, r, &a, &x, &Z);
            if (kg >= K) {
                /* not a topic at all: a disagreement whatever x is; the rest
                 * of the document is replayed with the oracle's own draw */
                out[2]++;
                if (*first_bad < 0) *first_bad = i;
                worst[0] = INFINITY;
                m[ko]++;
                continue;
            }
            if (ko == kg) { out[0]++; m[kg]++; continue; }
            /* distance from x to the x-values that yield kg */
            double sa = sigma_a[v];
            double dist = INFINITY;
            int64_t c0 = colptr[v];
            uint32_t j = mulhi(r[1], (uint32_t)(colptr[v + 1] - c0));
            int32_t ka = (r[2] < thr[c0 + j]) ? topic[c0 + j] : alias_topic[c0 + j];
            if (ka == kg) dist = x < sa ? 0.0 : x - sa;
            double lo = sa, c = sa;
            for (int32_t k = 0; k < K; k++) {
                double b = (double)phi[(size_t)k * V + v] * (double)m[k];
                if (b > 0.0) {
                    lo = c;
                    c += b;
                    if (k == kg) {
                        double dd = x < lo ? lo - x : (x >= c ? x - c : 0.0);
                        if (dd < dist) dist = dd;
                    }
                }
            }
            double rel = dist / Z;
            if (rel > worst[0]) worst[0] = rel;
            if (rel <= tol) out[1]++;
            else { out[2]++; if (*first_bad < 0) *first_bad = i; }
            m[kg]++;
        }
    }
    free(m);
}

/* ------------------------------------------------------------------------ */
/* Collapsed log joint (Griffiths & Steyvers 2004), fp64:                     */
/*  log p(w|z,beta) = K lgamma(V beta) - sum_k lgamma(n_k + V beta)            */
/*                    + sum_k sum_{v: n_kv>0} [lgamma(n_kv + beta) - lgamma(beta)]*/
/*  log p(z|alpha)  = D lgamma(A) - sum_d lgamma(N_d + A)                       */
/*                    + sum_d sum_{k: m_dk>0} [lgamma(m_dk + alpha_k) - lgamma(alpha_k)]*/
/*  with A = sum_k alpha_k.  Computed from z by counting, k-major then d-major.*/
/* ------------------------------------------------------------------------ */
double or_loglik(int64_t D, int32_t K, int32_t V, const int64_t *doc_off, const int32_t *words,
                 const uint16_t *z, const double *alpha, double beta, const double *beta_v)
{
    int32_t *n = (int32_t *)calloc((size_t)K * (size_t)V, sizeof(int32_t));
    int64_t *nk = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    int32_t *m = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    for (int64_t i = 0; i < doc_off[D]; i++) { n[(size_t)z[i] * V + words[i]]++; nk[z[i]]++; }
    /* with a vector beta_v: B = sum_v beta_v replaces V beta, and each
     * cell's term uses its word's beta_v */
    double Vb = (double)V * beta, lgb = lgamma(beta);
    if (beta_v) {
        Vb = 0.0;
        for (int32_t v = 0; v < V; v++) Vb += beta_v[v];
    }
    double word = (double)K * lgamma(Vb);
    for (int32_t k = 0; k < K; k++) {
        word -= lgamma((double)nk[k] + Vb);
        for (int32_t v = 0; v < V; v++) {
            int32_t c = n[(size_t)k * V + v];
            if (c > 0) word += beta_v ? lgamma((double)c + beta_v[v]) - lgamma(beta_v[v]) : lgamma((double)c + beta) - lgb;
        }
    }
    double A = 0.0;
    for (int32_t k = 0; k < K; k++) A += alpha[k];
    double doc = 0.0;
    for (int64_t d = 0; d < D; d++) {
        memset(m, 0, sizeof(int32_t) * (size_t)K);
        for (int64_t i = doc_off[d]; i < doc_off[d + 1]; i++) m[z[i]]++;
        double s = lgamma(A) - lgamma((double)(doc_off[d + 1] - doc_off[d]) + A);
        for (int32_t k = 0; k < K; k++)
            if (m[k] > 0) s += lgamma((double)m[k] + alpha[k]) - lgamma(alpha[k]);
        doc += s;
    }
    free(n); free(nk); free(m);
    return word + doc;
}

/* ------------------------------------------------------------------------ */
/* Fold-in of one new document against a fixed Phi.                          */
/* Tokens whose word is out of range or has an empty Phi column are dropped.  */
/* Kept tokens keep their position p in the request.  Initial topics          */
/* z_p = mulhi(r0 of ctr (p, req, 0, FOLDIN_INIT), K); then S sweeps of the    */
/* token draw with ctr (p, req, s, FOLDIN_Z), s = 1..S; after every sweep s > */
/* burn_in the document-topic counts are accumulated.                         */
/*   theta_k = (acc_k / (S - burn_in) + alpha_k) / (N' + A)                    */
/*   loglik = sum_p ln phi[z_p][w_p] + lgamma(A) - lgamma(N' + A)              */
/*            + sum_k [lgamma(m_k + alpha_k) - lgamma(alpha_k)]  (final state) */
/* Returns the number of kept tokens; *dropped gets the others.              */
/* ------------------------------------------------------------------------ */
int32_t or_foldin(int32_t K, int32_t V, const float *phi, const int64_t *colptr, const uint16_t *topic,
                  const uint32_t *thr, const uint16_t *alias_topic, const double *sigma_a,
                  const double *alpha, uint64_t seed, uint32_t req, const int32_t *words, int32_t len,
                  int32_t S, int32_t burn_in, float *theta, double *loglik, int32_t *dropped,
                  uint16_t *z_final /* len entries or NULL; dropped tokens get 0xFFFF */)
{
    or_model M = {K, V, phi, colptr, topic, thr, alias_topic, sigma_a};
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len > 0 ? len : 1));
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len > 0 ? len : 1));
    int32_t *m = (int32_t *)calloc((size_t)K, sizeof(int32_t));
    int64_t *acc = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    int32_t nk = 0;
    for (int32_t p = 0; p < len; p++) {
        int32_t v = words[p];
        if (v < 0 || v >= V || colptr[v + 1] == colptr[v]) continue;
        pos[nk++] = p;
    }
    *dropped = len - nk;
    for (int32_t q = 0; q < nk; q++) {
        uint32_t r[4];
        draw4(seed, (uint32_t)pos[q], req, 0, TAG_FOLDIN_INIT, r);
        z[q] = (int32_t)mulhi(r[0], (uint32_t)K);
        m[z[q]]++;
    }
    for (int32_t s = 1; s <= S; s++) {
        for (int32_t q = 0; q < nk; q++) {
            int32_t v = words[pos[q]];
            m[z[q]]--;
            uint32_t r[4];
            draw4(seed, (uint32_t)pos[q], req, (uint32_t)s, TAG_FOLDIN_Z, r);
            int a;
            z[q] = draw_token(&M, v, m, r, &a, NULL, NULL);
            m[z[q]]++;
        }
        if (s > burn_in)
            for (int32_t k = 0; k < K; k++) acc[k] += m[k];
    }
    double A = 0.0;
    for (int32_t k = 0; k < K; k++) A += alpha[k];
    for (int32_t k = 0; k < K; k++)
        theta[k] = (float)(((double)acc[k] / (double)(S - burn_in) + alpha[k]) / ((double)nk + A));
    double ll = 0.0;
    for (int32_t q = 0; q < nk; q++) ll += log((double)phi[(size_t)z[q] * V + words[pos[q]]]);
    ll += lgamma(A) - lgamma((double)nk + A);
    for (int32_t k = 0; k < K; k++)
        if (m[k] > 0) ll += lgamma((double)m[k] + alpha[k]) - lgamma(alpha[k]);
    *loglik = ll;
    if (z_final) {
        for (int32_t p = 0; p < len; p++) z_final[p] = 0xFFFF;
        for (int32_t q = 0; q < nk; q++) z_final[pos[q]] = (uint16_t)z[q];
    }
    free(pos); free(z); free(m); free(acc);
    return nk;
}

/* ------------------------------------------------------------------------ */
/* Test hook: the law one token draw induces, by exhaustive enumeration of    */
/* the 2^24 values u24(r0) can take.  mass_b[k] gets the probability of k     */
/* from u values that fall in the b-part; *mass_a the total probability of    */
/* the a-part (whose split over topics is the alias table's law).            */
/* ------------------------------------------------------------------------ */
void or_token_pmf(int32_t K, int32_t V, const float *phi, const int64_t *colptr, const uint16_t *topic,
                  const uint32_t *thr, const uint16_t *alias_topic, const double *sigma_a, int32_t v,
                  const int32_t *m, double *mass_b, double *mass_a)
{
    or_model M = {K, V, phi, colptr, topic, thr, alias_topic, sigma_a};
    int64_t *cnt = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    int64_t na = 0;
    uint32_t r[4] = {0, 0, 0, 0};
    for (uint32_t u = 0; u < (1u << 24); u++) {
        r[0] = u << 8;
        int a;
        int32_t k = draw_token(&M, v, m, r, &a, NULL, NULL);
        if (a) na++; else cnt[k]++;
    }
    for (int32_t k = 0; k < K; k++) mass_b[k] = (double)cnt[k] / 16777216.0;
    *mass_a = (double)na / 16777216.0;
    free(cnt);
}

/* ------------------------------------------------------------------------ */
/* Held-out log-likelihood of a new document, log p(w_d | Phi, alpha), by the */
/* left-to-right algorithm of Wallach, Murray, Salakhutdinov and Mimno        */
/* (2009, "Evaluation methods for topic models"), which Section 4 uses for    */
/* the held-out comparison.  Tokens whose word is >= V or whose Phi column is */
/* empty are dropped (as in fold-in); the nk kept tokens are taken in order.  */
/* R independent particles; at step n (n = 0 .. nk-1) each particle first    */
/* redraws its topics z_q, q = 0 .. n-1, in order, each from the token        */
/* conditional of Section 3.5 given its other topics among the first n, then */
/* takes                                                                      */
/*   Z_n = sum_k phi_{k,w_n} (m_k + alpha_k) = sigma_a(w_n) + sigma_b(w_n)     */
/* over its topics z_<n (the normaliser of the conditional of token n), and   */
/* draws z_n from that conditional.  The estimate is                          */
/*   sum_n log( (1/R) sum_r Z_n^(r) / (n + A) ),  A = sum_k alpha_k.           */
/* Random numbers: particle r's draw of token q at step n uses Philox counter */
/* (q, n, req, LTR + 256 r) (q = n for the new token).  Zs (R x nk, or NULL)   */
/* receives every Z_n^(r).  Returns the estimate.                             */
/* ------------------------------------------------------------------------ */
double or_heldout_ltr(int32_t K, int32_t V, const float *phi, const int64_t *colptr, const uint16_t *topic,
                      const uint32_t *thr, const uint16_t *alias_topic, const double *sigma_a,
                      const double *alpha, uint64_t seed, uint32_t req, const int32_t *words, int32_t len,
                      int32_t R, double *Zs, int32_t *kept_out)
{
    or_model M = {K, V, phi, colptr, topic, thr, alias_topic, sigma_a};
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len > 0 ? len : 1));
    int32_t nk = 0;
    for (int32_t p = 0; p < len; p++) {
        int32_t v = words[p];
        if (v < 0 || v >= V || colptr[v + 1] == colptr[v]) continue;
        pos[nk++] = p;
    }
    *kept_out = nk;
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)(nk > 0 ? nk : 1));
    int32_t *m = (int32_t *)calloc((size_t)R * (size_t)K, sizeof(int32_t));
    double A = 0.0;
    for (int32_t k = 0; k < K; k++) A += alpha[k];
    double ll = 0.0;
    for (int32_t n = 0; n < nk; n++) {
        double sum = 0.0;
        for (int32_t r = 0; r < R; r++) {
            int32_t *zr = z + (size_t)r * nk;
            int32_t *mr = m + (size_t)r * K;
            uint32_t rr[4];
            int a;
            for (int32_t q = 0; q < n; q++) {
                mr[zr[q]]--;
                draw4(seed, (uint32_t)q, (uint32_t)n, req, TAG_LTR + ((uint32_t)r << 8), rr);
                zr[q] = draw_token(&M, words[pos[q]], mr, rr, &a, NULL, NULL);
                mr[zr[q]]++;
            }
            double Z;
            draw4(seed, (uint32_t)n, (uint32_t)n, req, TAG_LTR + ((uint32_t)r << 8), rr);
            zr[n] = draw_token(&M, words[pos[n]], mr, rr, &a, NULL, &Z);
            mr[zr[n]]++;
            if (Zs) Zs[(size_t)r * nk + n] = Z;
            sum += Z / ((double)n + A);
        }
        ll += log(sum / (double)R);
    }
    free(pos); free(z); free(m);
    return ll;
}
