/*
 * pulda.h -- C ABI of libpulda.so: the Polya-urn partially collapsed Gibbs
 * sampler for LDA (Terenin, Magnusson, Jonsson, Draper, "Polya Urn Latent
 * Dirichlet Allocation: a doubly sparse massively parallel sampler",
 * arXiv 1704.03581), on one AMD Instinct MI355X (gfx950).
 *
 * Model and notation (Section 1, Table 1): D documents, vocabulary V, K topics,
 * N tokens; word type v(i) and topic indicator z_i of token i; n : K x V
 * topic-word counts; m : D x K document-topic counts; alpha (1 x K) and beta
 * (symmetric scalar here) the Dirichlet priors.
 *
 * One sweep is Algorithm 2 (Section 3):
 *   Phi-step  phi_k ~ PPU(n_k + beta) for every topic k (Definition of the
 *             Poisson Polya urn, Section 3.3): gamma_kv ~ Pois(beta + n_kv),
 *             phi_kv = gamma_kv / sum_v gamma_kv; Pois(beta + l) by Walker alias
 *             tables for l <= L and by rounded Gaussian draws for l > L
 *             (Section 3.4);
 *   z-step    z_i drawn with P(z_i = k) propto phi_{k,v(i)} alpha_k +
 *             phi_{k,v(i)} m^{-i}_{d,k}, sequentially within each document,
 *             documents in parallel (Section 3.5: a-part from a per-word
 *             alias table, b-part summed over the smaller of the document's
 *             and the word's nonzero topics);
 *   counts    n and m rebuilt from z (Table 1: statistics of the current
 *             iteration).
 *
 * Random numbers come from Philox4x32-10 (Salmon et al., SC'11) keyed by the
 * model seed, with counters naming what is drawn (token index and sweep t,
 * or word, topic and t), so every result is a deterministic function of
 * (corpus, seed, state, t) and independent of the schedule.
 *
 * Conventions for every function below:
 *  - Every function returns a pulda_status.  Nothing aborts and no C++
 *    exception crosses the ABI.  pulda_last_error() gives a message for the
 *    last failure on the calling thread.
 *  - Argument errors are detected on the host before any launch; the call
 *    then changes no state (PULDA_ERR_INVALID_ARG).  Calls out of order (a
 *    z-step before init, a sweep before upload) return PULDA_ERR_STATE.
 *    HIP failures return PULDA_ERR_DEVICE.
 *  - "_dev" pointers are device (HBM) pointers owned by the caller; "_host"
 *    pointers are host memory, read or written before the call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it and the call returns without waiting, except where a function is
 *    documented as synchronising (it then waits for that stream).
 *  - The library allocates no device memory.  A plan (and a fold-in server)
 *    carves all its device buffers from one caller-owned workspace.  (A
 *    fold-in server holds pinned host staging buffers, see
 *    pulda_foldin_bind.)
 *  - One plan must not be used from two threads at the same time; distinct
 *    plans are independent.
 */
#ifndef PULDA_H
#define PULDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pulda_status;

enum {
    PULDA_OK = 0,
    PULDA_ERR_INVALID_ARG = -1,  /* bad argument; nothing was launched */
    PULDA_ERR_STATE = -2,        /* call out of order */
    PULDA_ERR_DEVICE = -3,       /* a HIP call or kernel launch failed */
    PULDA_ERR_NO_MEMORY = -4,    /* the bound workspace is smaller than required */
    PULDA_ERR_CAPACITY = -5,     /* fold-in: no free slot or arena space now; retry later */
    PULDA_ERR_CORPUS = -6        /* corpus content invalid (offsets, word ids, length) */
};

/* Message of the last failure on the calling thread ("" if none). */
const char *pulda_last_error(void);
/* Library version string. */
const char *pulda_version(void);

/* ------------------------------------------------------------------------ */
/* Model and plan                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t K;               /* topics, 1 <= K <= 4096 */
    int32_t V;               /* vocabulary size, >= 1; V * (K rounded up to 64) < 2^30 */
    double beta;             /* symmetric prior on each phi_k (Table 1), > 0 */
    double alpha;            /* symmetric prior on each theta_d, > 0; used when alpha_k is NULL */
    const double *alpha_k;   /* optional host vector of K priors alpha_k > 0 (copied), or NULL */
    int32_t L;               /* Poisson alias tables for rates beta + l, 1 <= l <= L (Section 3.4); 1..1000 */
    uint64_t seed;           /* Philox key */
    const double *beta_v;    /* optional host vector of V priors beta_v in (0, 16] (copied; beta is then
                                ignored), or NULL for the symmetric beta in (0, 16].  The paper's beta is a
                                V-vector (Section 3.2); with per-word priors the Polya-urn Phi-step draws
                                a counted cell's Pois(beta_v + n_kv) as Pois(n_kv) (alias tables of integer
                                rates, a rounded Gaussian above L) plus the cell's prior mark, the
                                zero-truncated Pois(beta_v) value the column's jumps at rate beta_v give
                                every marked cell, counted or not: the same law.  The Dirichlet Phi-step
                                uses shapes beta_v + n_kv and the log joint sum_v beta_v and
                                lgamma(n_kv + beta_v). */
} pulda_model_desc;

typedef struct pulda_plan pulda_plan;

/* Create a plan for a corpus of D documents and N tokens (D >= 0, N >= 0,
 * N < 2^40).  *out receives the plan (host object, freed by
 * pulda_plan_destroy). */
pulda_status pulda_plan_create(const pulda_model_desc *desc, int64_t D, int64_t N, pulda_plan **out);

/* Bytes of device workspace the plan needs (256-byte aligned start). */
pulda_status pulda_plan_workspace_bytes(const pulda_plan *plan, int64_t *bytes);

/* Bind a caller-owned device workspace of `bytes` bytes.  It must stay
 * allocated and untouched by the caller until the plan is destroyed.
 * PULDA_ERR_NO_MEMORY if bytes is below pulda_plan_workspace_bytes. */
pulda_status pulda_plan_bind(pulda_plan *plan, void *workspace_dev, int64_t bytes);

void pulda_plan_destroy(pulda_plan *plan);

/* ------------------------------------------------------------------------ */
/* Corpus and state                                                          */
/* ------------------------------------------------------------------------ */

/* Attach the corpus (Section 1): documents as CSR, doc_off_dev[D+1] (int64,
 * doc_off[0] = 0, non-decreasing, doc_off[D] = N) and words_dev[N] (int32 word
 * ids in [0, V)); tokens of a document are sampled in this stored order.
 * Both arrays stay owned by the caller and must stay valid and unmodified
 * while the plan uses them.  Synchronises: validates the content on the
 * device (PULDA_ERR_CORPUS for bad offsets, word ids, or a document longer
 * than 65535 tokens) and orders documents by length for the z-step
 * schedule.  When K <= 256 it also counts the words of the first 8M tokens
 * on the host and keeps the most frequent ones (as many as 4096 / K), whose
 * count increments the z-step gathers per block before adding them to n
 * (the counts are the same). */
pulda_status pulda_corpus_upload(pulda_plan *plan, const int64_t *doc_off_dev, const int32_t *words_dev,
                                 void *stream);

/* Initial state: z0_dev[N] (uint16 topics < K, copied) or, with NULL, z_i
 * uniform on {0..K-1} from Philox counter (i, 0, tag 0).  Rebuilds n. */
pulda_status pulda_init(pulda_plan *plan, const uint16_t *z0_dev, void *stream);

/* Replace z by z_dev[N] (uint16, < K; copied) and rebuild n: resume from a
 * checkpoint or teacher-force a state. */
pulda_status pulda_set_z(pulda_plan *plan, const uint16_t *z_dev, void *stream);

/* Copy z (uint16[N]) into z_dev. */
pulda_status pulda_get_z(const pulda_plan *plan, uint16_t *z_dev, void *stream);

/* Replace the topic-word counts by n_dev[V*K] (int32 >= 0, word-major:
 * n[v*K + k]).  Used to build a Phi from counts held elsewhere (a serving
 * model) without a corpus. */
pulda_status pulda_set_counts(pulda_plan *plan, const int32_t *n_dev, void *stream);

/* ------------------------------------------------------------------------ */
/* Algorithm 2                                                               */
/* ------------------------------------------------------------------------ */

/* Phi-step of sweep t (t >= 1) from the current counts n: draws gamma, the
 * row sums S_k, phi = fp32(gamma / S_k) (fp64 quotient), the CSC of Phi's
 * nonzeros by word, each word's alias table over alpha_k phi_kv and
 * sigma_a(v) = sum_k alpha_k phi_kv (Sections 3.3-3.5).  A row with S_k = 0
 * stays empty (the PPU is defined for a nonzero sum only). */
pulda_status pulda_phi_step(pulda_plan *plan, uint32_t t, void *stream);

/* z-step of sweep t with the current Phi, followed by the count rebuild of
 * n.  A token whose word has an empty Phi column (0/0 conditional) keeps its
 * topic and is counted in pulda_sweep_stats.degenerate_tokens. */
pulda_status pulda_z_step(pulda_plan *plan, uint32_t t, void *stream);

/* n_sweeps sweeps t_first, t_first+1, ...: Phi-step, z-step, and the log
 * joint of each sweep's state.  If ll_host is non-NULL it receives
 * n_sweeps values and the call synchronises; otherwise it is asynchronous.
 * With graph replay enabled (pulda_set_graph) one captured sweep is
 * replayed with a device-side sweep counter. */
pulda_status pulda_sweep(pulda_plan *plan, uint32_t t_first, int32_t n_sweeps, double *ll_host, void *stream);

/* Collapsed log joint log p(w | z, beta) + log p(z | alpha) of the current
 * state (the per-iteration log-posterior trace of Section 4), fp64.
 * Synchronises. */
pulda_status pulda_loglik(pulda_plan *plan, double *ll_host, void *stream);

/* ------------------------------------------------------------------------ */
/* Counts and Phi export / import                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *n_colptr_dev;   /* [V+1] */
    uint16_t *n_topic_dev;   /* [nnz_n] ascending within each word */
    int32_t *n_count_dev;    /* [nnz_n] */
    int64_t *nk_dev;         /* [K] n_k = sum_v n_kv */
    int64_t *m_rowptr_dev;   /* [D+1] */
    uint16_t *m_topic_dev;   /* [nnz_m] ascending within each document */
    int32_t *m_count_dev;    /* [nnz_m] */
} pulda_counts_view;

/* Numbers of nonzeros of n and m for the current z.  Synchronises. */
pulda_status pulda_counts_sizes(pulda_plan *plan, int64_t *nnz_n, int64_t *nnz_m, void *stream);

/* Write n (CSC by word) and m (CSR by document) of the current z into the
 * caller's buffers, sized by pulda_counts_sizes.  Synchronises. */
pulda_status pulda_counts(pulda_plan *plan, const pulda_counts_view *out, void *stream);

/* Dense counts: n_dev[V*K] (int32, word-major) and nk_dev[K] (int64); either
 * may be NULL. */
pulda_status pulda_get_counts_dense(pulda_plan *plan, int32_t *n_dev, int64_t *nk_dev, void *stream);

typedef struct {
    int64_t *colptr_dev;        /* [V+1] */
    uint16_t *topic_dev;        /* [nnz] ascending within each word */
    int32_t *gamma_dev;         /* [nnz] Poisson draws (export only; may be NULL) */
    float *phi_dev;             /* [nnz] */
    uint32_t *alias_thr_dev;    /* [nnz] keep entry e when r < thr (0xFFFFFFFF: always) */
    uint16_t *alias_topic_dev;  /* [nnz] topic drawn otherwise */
    double *sigma_a_dev;        /* [V] */
    int64_t *S_dev;             /* [K] row sums of gamma (export only; may be NULL) */
} pulda_phi_view;

/* The Phi-step that pulda_phi_step and pulda_sweep run (default
 * PULDA_PHI_POLYA_URN).  Either way the z-step that follows is the same.
 *   PULDA_PHI_POLYA_URN: Algorithm 2's step, phi_k ~ PPU(n_k + beta): Poisson
 *     draws gamma_kv ~ Pois(beta + n_kv) (alias tables for n_kv <= L, a
 *     rounded Gaussian above), phi_kv = fp32(gamma_kv / S_k) (Section 3.4).
 *   PULDA_PHI_DIRICHLET: Algorithm 1's step, phi_k ~ Dir(n_k + beta) by the
 *     Gamma representation (Section 3.3): gamma_kv ~ G(beta + n_kv, 1) by
 *     Marsaglia and Tsang's method (the one Section 3.4 names; boost for
 *     shapes below 1), S_k = sum_v gamma_kv in fp64 (fixed order: ascending
 *     within blocks of 256 words, then over the blocks), phi_kv =
 *     fp32(gamma_kv / S_k); cells whose fp32 phi is below 2^-126 (zero or
 *     subnormal) are zero, so Phi holds about K * V nonzeros and costs that
 *     much memory traffic in the z-step.  Philox counter of attempt j of cell
 *     (k, v) at sweep t: (v, k, t, 6 + 256 j).
 * Invalid method: PULDA_ERR_INVALID_ARG.  A captured sweep graph is rebuilt. */
enum { PULDA_PHI_POLYA_URN = 0, PULDA_PHI_DIRICHLET = 1 };
pulda_status pulda_set_phi_method(pulda_plan *plan, int32_t method);

/* After a Dirichlet Phi-step: its Gamma draws gamma_dev[V*K] (fp64,
 * word-major: gamma_dev[v*K + k]) and row sums S_dev[K] (fp64); either may be
 * NULL.  PULDA_ERR_STATE when the last Phi-step was not a Dirichlet one. */
pulda_status pulda_get_gamma_dense(pulda_plan *plan, double *gamma_dev, double *S_dev, void *stream);

/* Number of nonzeros of Phi after the last Phi-step.  Synchronises. */
pulda_status pulda_phi_nnz(pulda_plan *plan, int64_t *nnz, void *stream);
/* Write Phi (CSC by word), its alias tables and sigma_a. */
pulda_status pulda_get_phi(pulda_plan *plan, const pulda_phi_view *out, void *stream);
/* Load Phi from the caller (e.g. a trained model for fold-in); gamma_dev and
 * S_dev are ignored.  colptr_dev[V] must not exceed K * V. */
pulda_status pulda_set_phi(pulda_plan *plan, const pulda_phi_view *in, void *stream);

/* ------------------------------------------------------------------------ */
/* Statistics, schedule, graph replay                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    /* z-step counters, summed over the z-steps since the previous
     * pulda_stats call (which resets them) */
    int64_t degenerate_tokens;  /* tokens with an empty Phi column (kept their topic) */
    int64_t sum_J;              /* sum over tokens of min(K_d^{-i}, K_v^Phi): the work of the
                                   doubly sparse b-sum (computational complexity, Section 3.6) */
    int64_t sum_A;              /* tokens drawn from the a-part */
    int64_t z_steps;            /* z-steps counted */
    /* last Phi-step */
    int64_t nnz_phi;
    int64_t empty_rows;         /* topics with S_k = 0 */
    /* with timing on (pulda_set_timing): milliseconds between hipEvents
     * recorded on the caller's stream around each Phi-step, each z-step
     * kernel and each log-joint evaluation since the previous call, and
     * how many of each */
    double ms_phi, ms_z, ms_ll;
    int64_t n_phi, n_z, n_ll;
    /* sum_J over the tokens whose b-terms were computed: a token whose
     * a-part is certain from sigma_a and a bound on sigma_b (decided when it
     * is staged) counts in sum_J but not here */
    int64_t sum_J_b;
    /* z-step draws whose fp32 b-part left the decision to the fp64 one (y
     * within its rounding bound of a boundary) */
    int64_t fallback_draws;
} pulda_sweep_stats;

/* Read (and restart) the counters above.  Synchronises. */
pulda_status pulda_stats(pulda_plan *plan, pulda_sweep_stats *out, void *stream);

/* Record hipEvents around every phase (1) or not (0).  While on, pulda_sweep
 * runs eagerly (no graph replay). */
pulda_status pulda_set_timing(pulda_plan *plan, int32_t enable);

/* z-step schedule: documents are ordered by decreasing length and split
 * into n_buckets length buckets; bucket b holds documents with length >=
 * min_len[b] (min_len decreasing, last 0) and is processed by groups of
 * group[b] lanes (1, 8, 16, 32 or 64) with docs_per_item[b] documents per
 * work item (a multiple of 64 / group).  Group 1 runs one document per lane
 * (its b-sum is the sequential ascending sum) and takes documents shorter
 * than 128 tokens (256 when K <= 127); groups of 8 take documents shorter than 256
 * tokens; a
 * work item whose group would not fit runs on a larger group size.  A token's b-terms (Section 3.5) are summed
 * over the word's Phi column or over the document's topics; a group prefers
 * the column when K_v <= side_ratio[b] * K_d (side_ratio NULL: all 1, the
 * smaller side) and a wave takes the document side when any of its groups
 * prefers it.  Results do not depend on the schedule except through fp64
 * rounding order. */
pulda_status pulda_set_schedule(pulda_plan *plan, int32_t n_buckets, const int32_t *min_len_host,
                                const int32_t *group_host, const int32_t *docs_per_item_host,
                                const int32_t *side_ratio_host);
pulda_status pulda_get_schedule(const pulda_plan *plan, int32_t cap, int32_t *n_buckets, int32_t *min_len_host,
                                int32_t *group_host, int32_t *docs_per_item_host, int32_t *side_ratio_host);

/* Time each candidate group size (1, 8, 16, 32, 64) and side ratio (1, 4, 16) on
 * each bucket (z-step at sweep t, reps repetitions, current Phi) and keep the
 * fastest; then time the whole z-step, as a sweep launches it, with each
 * bucket moved into every other bucket's group and side ratio, and keep a
 * move that makes it faster (a bucket alone in its kernel may run after the
 * others).  Restores z and n.  Synchronises. */
pulda_status pulda_autotune(pulda_plan *plan, uint32_t t, int32_t reps, void *stream);

/* In pulda_sweep, let the z-step write each document's term of the log
 * joint from the counts it already holds (1, default; symmetric alpha only)
 * or recount them from z in a separate pass (0).  Same value either way up
 * to fp64 summation order. */
pulda_status pulda_set_fused_loglik(pulda_plan *plan, int32_t enable);

/* Enable (1) or disable (0) replaying a captured sweep in pulda_sweep. */
pulda_status pulda_set_graph(pulda_plan *plan, int32_t enable);

/* ------------------------------------------------------------------------ */
/* Fold-in serving (theta inference for new documents against a fixed Phi)  */
/* ------------------------------------------------------------------------ */
/* A request is one new document.  Tokens whose word is out of range or has
 * an empty Phi column are dropped and counted.  The kept tokens start from
 * topics drawn with Philox counter (p, request_id, 0, tag 4) and run `sweeps`
 * sweeps of the z-step's token draw with counters (p, request_id, s, tag 5),
 * p the token's position in the request; the topic counts are averaged over
 * sweeps after `burn_in`:
 *   theta_k = (mean m_k + alpha_k) / (kept + sum alpha),
 * and the log-likelihood of the final state is
 *   sum_p ln phi[z_p][w_p] + ln Gamma(A) - ln Gamma(kept + A)
 *   + sum_k [ln Gamma(m_k + alpha_k) - ln Gamma(alpha_k)].
 * Results depend only on (Phi, seed, request_id, words): they are the same
 * whether a request runs alone or among others.  request_id must be unique
 * among requests in flight. */
typedef struct {
    int32_t sweeps;       /* >= 1 */
    int32_t burn_in;      /* 0 <= burn_in < sweeps */
    int32_t max_slots;    /* requests resident at once */
    int32_t arena_tokens; /* device token capacity shared by resident requests */
    int32_t max_len;      /* longest accepted request, <= arena_tokens, <= 65535 */
    int32_t group;        /* lanes per request: 16, 32 or 64 */
    uint64_t seed;
} pulda_foldin_desc;

typedef struct pulda_foldin pulda_foldin;

typedef struct {
    uint32_t request_id;
    int32_t kept;
    int32_t dropped;
    int32_t pad;
    double loglik;
} pulda_foldin_result;

/* Create a server over the plan's current Phi (which it reads; the plan
 * must outlive the server and its Phi must not change meanwhile). */
pulda_status pulda_foldin_create(const pulda_plan *model, const pulda_foldin_desc *desc, pulda_foldin **out);
pulda_status pulda_foldin_workspace_bytes(const pulda_foldin *f, int64_t *bytes);
/* Bind the caller's device workspace.  The first bind also allocates the
 * server's pinned host staging (arena_tokens * 4 bytes for request words and
 * two copies of the slot table), through which every host-to-device copy of
 * submit and step goes, so no copy reads the caller's memory after the call
 * returns; pulda_foldin_destroy frees it.  PULDA_ERR_NO_MEMORY if the
 * workspace is too small or the staging cannot be allocated. */
pulda_status pulda_foldin_bind(pulda_foldin *f, void *workspace_dev, int64_t bytes);
void pulda_foldin_destroy(pulda_foldin *f);

/* Admit a request: copies words_host[len] into a free slot's arena region.
 * PULDA_ERR_CAPACITY when no slot or no contiguous arena space is free now
 * (the request is not admitted; retry after a poll).  PULDA_ERR_INVALID_ARG
 * if len > max_len or len < 0. */
pulda_status pulda_foldin_submit(pulda_foldin *f, uint32_t request_id, const int32_t *words_host, int32_t len,
                                 void *stream);

/* Advance every resident request by up to `draws` token draws in one launch
 * (asynchronous).  A request resumes where its previous step stopped (sweep
 * and token within it; the progress is kept on the device), so a step takes
 * about the same time for long and short requests.  Results do not depend
 * on how a request's draws are split into steps. */
pulda_status pulda_foldin_step(pulda_foldin *f, int32_t draws, void *stream);

/* Collect finished requests (at most cap): results into out[], theta into
 * theta_host[cap * K] (row j for out[j]); frees their slots.  Reads the
 * requests' progress from the device after every step launched on `stream`.
 * Synchronises the stream. */
pulda_status pulda_foldin_poll(pulda_foldin *f, pulda_foldin_result *out, float *theta_host, int32_t cap,
                               int32_t *n_done, void *stream);

/* As pulda_foldin_poll, for the requests finished by the step before the
 * latest pulda_foldin_step: the copies run on the server's own stream behind
 * that step only, so the latest step keeps running meanwhile.  A serving
 * loop that launches step s, then collects step s-1's results and admits new
 * requests while step s runs keeps the GPU busy through its own host work.
 * Step s skips the requests that finished before it (their results stay as
 * written), and a request finished by step s is collected by the poll after
 * step s+1 (one more step, of no work for it, may be needed at the end).
 * Nothing to collect before the second step.  Synchronises the server's
 * stream only. */
pulda_status pulda_foldin_poll_previous(pulda_foldin *f, pulda_foldin_result *out, float *theta_host, int32_t cap,
                                        int32_t *n_done);

/* Resident and free slot counts. */
pulda_status pulda_foldin_occupancy(const pulda_foldin *f, int32_t *resident, int32_t *free_slots,
                                    int32_t *free_tokens);

/* ------------------------------------------------------------------------ */
/* Held-out log-likelihood of new documents                                  */
/* ------------------------------------------------------------------------ */
/* log p(w_d | Phi, alpha) of D documents by the left-to-right algorithm of
 * Wallach, Murray, Salakhutdinov and Mimno (2009), the estimator the paper's
 * Section 4 uses for its held-out comparison, against the plan's current Phi
 * (a Phi-step's or pulda_set_phi's).  Tokens whose word is >= V or whose Phi
 * column is empty are dropped.  Each of R particles, at step n (over the kept
 * tokens in order), redraws its topics of tokens 0..n-1 in order from the
 * token conditional of Section 3.5 (phi_kv (alpha_k + m_k), the fold-in and
 * z-step draw), then takes Z_n = sum_k phi_{k,w_n} (m_k + alpha_k) over its
 * topics of tokens 0..n-1 and draws z_n.  ll_dev[d] = sum_n log((1/R)
 * sum_r Z_n^(r) / (n + A)), A = sum_k alpha_k.  The cost is about R n^2 / 2
 * token draws per document of n tokens.
 *   doc_off_dev[D+1], words_dev[N]: the documents (device, CSR; each at most
 *     65535 tokens; the offsets are copied to the host and checked:
 *     PULDA_ERR_CORPUS).
 *   req_dev[D]: request ids; particle r's draw of token q at step n uses
 *     Philox counter (q, n, req, 7 + 256 r) under seed.
 *   particles in [1, 2^24); group: lanes per particle (16, 32, 64).
 *   workspace_dev: pulda_heldout_workspace_bytes(model, D, N, particles) bytes,
 *     256-byte aligned, caller-owned.
 *   ll_dev[D] (fp64) and kept_dev[D] (kept tokens) are written; Z_dev (R*N
 *     fp64, or NULL) receives Z_n^(r) of document d at doc_off[d]*R + r*N_d + n.
 * Documents are processed longest first (the order is computed on the host
 * and copied into the workspace).  The call synchronises the stream for the
 * offset check and for that copy; the kernels are then stream-ordered. */
pulda_status pulda_heldout_workspace_bytes(const pulda_plan *model, int64_t D, int64_t N, int32_t particles,
                                           int64_t *bytes);
pulda_status pulda_heldout_loglik(const pulda_plan *model, int64_t D, const int64_t *doc_off_dev,
                                  const int32_t *words_dev, const uint32_t *req_dev, int32_t particles, int32_t group,
                                  uint64_t seed, void *workspace_dev, int64_t workspace_bytes, double *ll_dev,
                                  int32_t *kept_dev, double *Z_dev, void *stream);

/* The held-out estimate for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * pulda_heldout_loglik with the same arguments and results but no workspace.
 * Its scratch is the library's own array of
 * PULDA_HELDOUT_NOALLOC_SCRATCH_BYTES bytes on each GPU it runs on (held
 * until the process ends; its address is looked up on the first call on
 * each device).  It needs pulda_heldout_workspace_bytes(model, D, N,
 * particles) bytes; larger calls return PULDA_ERR_NO_MEMORY and launch
 * nothing.  The call allocates no device memory.  Every call on one GPU
 * shares that GPU's scratch: calls that overlap in time on one GPU (other
 * streams or threads) race and must be serialised by the caller.  Each
 * call writes every scratch word it reads, so nothing carries over from the
 * previous call. */
#define PULDA_HELDOUT_NOALLOC_SCRATCH_BYTES (32ll << 20)
pulda_status pulda_heldout_loglik_noalloc(const pulda_plan *model, int64_t D, const int64_t *doc_off_dev,
                                          const int32_t *words_dev, const uint32_t *req_dev, int32_t particles,
                                          int32_t group, uint64_t seed, double *ll_dev, int32_t *kept_dev,
                                          double *Z_dev, void *stream);

/* The plain per-document sampler: runs one request alone, all sweeps in one
 * launch, and waits for it (uses the server's workspace; the server must be
 * empty).  Same results as the batched path. */
pulda_status pulda_foldin_run_one(pulda_foldin *f, uint32_t request_id, const int32_t *words_host, int32_t len,
                                  float *theta_host, pulda_foldin_result *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PULDA_H */
