// Internal declarations shared by the kernels and the C ABI (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

namespace pulda {

// device buffers of one model, carved from the caller's workspace
struct DevModel {
    int32_t K, V, L;
    double beta;
    uint32_t key0, key1;
    const double *alpha;          // [K]
    // counts of the current state (word-major dense: n[v*K + k])
    int32_t *n;
    unsigned long long *nk;       // [K]
    // Phi-step
    int32_t *gam;                 // [V*K] Poisson draws, word-major dense
    unsigned long long *S;        // [K] row sums
    float *phid;                  // [V*K] dense phi, word-major
    // 16-bit copy of gam for the z-step's document-side gathers, word-major
    // with row stride ks16 (K rounded up to 64: 128-byte aligned rows).
    // phi_kv is recovered as fp32(gam_kv * R_k) with R_k = RN64(1 / S_k):
    // for gam < 2^16 and S_k < 2^27 no fp32 rounding midpoint lies within
    // the product's error of gam / S_k, so this equals fp32(RN64(gam / S_k))
    // bit for bit.  Every other nonzero cell (gam >= 0xFFFF, S_k >= 2^27, or
    // a Phi loaded from values) holds 0xFFFF and is read from phid.
    uint16_t *g16;
    int32_t ks16;
    double *Rd;                   // [K] RN64(1 / S_k) (0 for an empty row)
    // Algorithm 1's Phi-step (phi_k ~ Dir(n_k + beta)): Gamma draws
    // (word-major dense, fp64), their row sums, and per-block partial sums
    double *gamd;                 // [V*K]
    double *Sd;                   // [K]
    double *dpart;                // [ceil(V / ROWSUM_COLS) * K]
    int32_t phi_method;           // of the last Phi-step: 0 Polya urn, 1 Dirichlet
    int32_t *colcnt;              // [V]
    int32_t *colptr;              // [V+1]
    uint16_t *ctopic;             // [cap] CSC by word, ascending topic
    float *cphi;                  // [cap]
    uint32_t *ckg;                // [cap] topic | 16-bit draw << 16 (as g16)
    uint64_t *calias;             // [cap] thr | topic << 32 | alias_topic << 48
    double *sigma_a;              // [V]
    float *phimax;                // [V] the largest phi of each word's column
    // per word, what a z-step token needs of its word in one 16-byte load:
    // {first CSC entry, column length, fp32(sigma_a), phimax} (as bits)
    uint4 *wrec;                  // [V]
    // the corpus's most frequent words, whose count increments the z-step
    // gathers per block in LDS when K is small (hot[v]: the word's index
    // among them, or -1; hot_word[h]: the word of index h)
    int32_t *hot;                 // [V]
    int32_t *hot_word;            // [HOT_MAX]
    int32_t n_hot;
    const uint64_t *pois;         // Poisson alias tables, thr | x_alias << 32
    const int32_t *pois_off;      // [L+2]
    // per-word priors (null: the symmetric beta); zero-truncated
    // Pois(beta_v) thresholds floor(2^32 P(X <= x | X >= 1)), x = 1.., one row
    // per word in ztp_tab from ztp_off (null: one row of ztp_n for beta)
    const double *beta_v;         // [V]
    const uint32_t *ztp_tab;
    const int32_t *ztp_off;       // [V+1]
    int32_t ztp_n;
    double beta_sum;              // sum_v beta_v (V beta for the symmetric prior)
    // log-joint terms for integer counts x < LG_TABLE:
    //   lg_beta[x] = lgamma(x + beta) - lgamma(beta),
    //   lg_alpha[x] = lgamma(x + alpha) - lgamma(alpha) (symmetric alpha only, else null),
    //   lg_A[x] = lgamma(A) - lgamma(x + A), A = sum_k alpha_k
    const double *lg_beta, *lg_alpha, *lg_A;
    const uint32_t *tptr;         // sweep number t, read on the device
    long long *scratch;           // scan scratch: ceil(max(V, D) / 1024) + 2 entries
};

struct DevCorpus {
    int64_t D, N;
    const int64_t *doc_off;
    const int32_t *words;
    uint16_t *z;
    const int32_t *doc_order;     // documents by decreasing length
};

// a unit of z-step work: `count` documents of doc_order starting at `first`,
// processed by groups of `group` lanes; the b-terms of a token are taken
// from the word's Phi column when K_v <= side_ratio * K_d, else from the
// document's topics (which side is walked changes cost, not the result)
struct WorkItem {
    int32_t first, count, group, side_ratio;
};

// slots per lane of the z-step's windowed topic list (groups of 16: 8,
// else 4)
inline int32_t z_window(int32_t group) { return group == 16 ? 8 : 4; }

// LDS layout of one z-step class (group size, count width): per group a
// count table (K counters of 1 or 2 bytes, rounded to 16 bytes) and the
// document's topic list (u16; min(K, 255) entries for documents shorter
// than 256 tokens, else K, and at least W slots per lane and W more, for
// the list's windows of W = z_window(group) slots, 16-byte aligned), 64/G
// groups per wave, and the block's copy of R_k (K floats) first
struct ZLayout {
    int32_t m_bytes, group_bytes, wave_bytes, r_bytes;
};

inline ZLayout z_layout(int32_t group, bool narrow, int32_t K)
{
    ZLayout L;
    const int32_t W = z_window(group);
    L.m_bytes = (K * (narrow ? 1 : 2) + 15) / 16 * 16;
    int32_t lcap = narrow ? (K < 255 ? K : 255) : K;
    if (lcap < W * group + W) lcap = W * group + W;
    L.group_bytes = L.m_bytes + (lcap * 2 + 15) / 16 * 16;
    L.wave_bytes = ((64 / group) * L.group_bytes + 15) / 16 * 16;
    L.r_bytes = (K * 4 + 15) / 16 * 16;
    return L;
}

// LDS for the per-block counts of the frequent words (hot words) and the
// fewest such words worth it
constexpr int32_t HOT_BYTES = 16384;
constexpr int32_t HOT_MIN = 16;
constexpr int32_t HOT_MAX = HOT_BYTES / 4;

// ST_TOKENS counts z-step launches since the last statistics read
constexpr int32_t LG_TABLE = 65536;

// work-item queues of a z-step: one atomic counter per class, cleared by
// launch_z_prepare
constexpr int32_t Z_QUEUES = 16;

enum StatIndex { ST_DEGENERATE = 0, ST_SUM_J = 1, ST_SUM_A = 2, ST_NNZ_PHI = 3, ST_EMPTY_ROWS = 4, ST_TOKENS = 5,
                 ST_SUM_JB = 6, ST_FALLBACK = 7, ST_COUNT = 8 };

// launchers (stream-ordered; return the launch status)
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count, hipStream_t s);
hipError_t launch_validate(const DevCorpus &c, int32_t V, int32_t *err, hipStream_t s);
hipError_t launch_init_z(const DevCorpus &c, int32_t K, uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t launch_count_rebuild(const DevCorpus &c, const DevModel &m, hipStream_t s);
hipError_t launch_row_sums(const int32_t *dense, int32_t V, int32_t K, unsigned long long *out, hipStream_t s);
hipError_t launch_phi_step(const DevModel &m, unsigned long long *stats, hipStream_t s);
// Algorithm 1's Phi-step into the same Phi tables (m.phi_method must be 1)
hipError_t launch_phi_step_dirichlet(const DevModel &m, unsigned long long *stats, hipStream_t s);
constexpr int32_t ROWSUM_COLS = 256;      // words per block of the row-sum kernels
// z-step: launch_z_prepare clears n and the Z_QUEUES work queues; then one
// persistent kernel per work-item class (group size 8 to 64 and count
// width, or one document per lane) over that class's items.
// With ll_doc non-null (symmetric alpha) the z-step also writes each
// document's term of the log joint for the state it leaves.
hipError_t launch_z_prepare(const DevModel &m, int32_t *queues, unsigned long long *stats, hipStream_t s);
// narrow: 8-bit document-topic counts (every document of the items is
// shorter than 256 tokens; group 8, 16 or 32).  The grid is as many blocks
// as n_cu compute units hold at once.
hipError_t launch_z_class(const DevCorpus &c, const DevModel &m, int32_t group, bool narrow, const WorkItem *items,
                          int32_t n_items, int32_t n_cu, int32_t *queue, unsigned long long *stats,
                          double *ll_doc, hipStream_t s);
// log joint of the current state; with ll_doc non-null the document terms
// are taken from it (written by the z-step) instead of recounted from z
hipError_t launch_loglik(const DevCorpus &c, const DevModel &m, double *partials, int32_t n_part_words,
                         int32_t n_part_docs, const double *ll_doc, double *out, double *hist,
                         const uint32_t *hist_idx, hipStream_t s);
hipError_t launch_advance(uint32_t *tptr, uint32_t *hist_idx, hipStream_t s);
hipError_t launch_n_colcount(const DevModel &m, int64_t *cnt, hipStream_t s);
// rebuild the per-word records from colptr, sigma_a and phimax
hipError_t launch_word_records(const DevModel &m, hipStream_t s);
hipError_t launch_export_phi(const DevModel &m, int64_t *colptr64, uint16_t *topic, int32_t *gam_e, float *phi_e,
                             uint32_t *thr, uint16_t *alias_topic, hipStream_t s);
hipError_t launch_import_phi(const DevModel &m, const int64_t *colptr64, const uint16_t *topic, const float *phi_e,
                             const uint32_t *thr, const uint16_t *alias_topic, hipStream_t s);
hipError_t launch_counts_csc(const DevModel &m, const int64_t *colptr64, uint16_t *topic, int32_t *cnt,
                             int32_t *colcnt_scratch, hipStream_t s);
hipError_t launch_counts_m(const DevCorpus &c, int32_t K, int64_t *rowcnt_or_ptr, uint16_t *topic, int32_t *cnt,
                           int pass, hipStream_t s);
hipError_t launch_check_u16_below(const uint16_t *x, int64_t n, uint32_t limit, int32_t *err, hipStream_t s);
hipError_t launch_check_phi(const int64_t *colptr, int32_t V, const uint16_t *topic, const uint16_t *alias_topic,
                            uint32_t K, int32_t *err, hipStream_t s);
hipError_t launch_scan_i64(const int64_t *in, int64_t *out_excl, int64_t n, long long *scratch, hipStream_t s);

// fold-in
// host-written control of a resident request
struct FoldSlot {
    int32_t arena_off;  // first token of the slot's region in the arena
    int32_t len;        // request length
    uint32_t req;       // request id
    int32_t fresh;      // 1 on the request's first step (drop tokens, draw initial topics)
    int32_t budget;     // token draws to run in this step
    int32_t pad[3];
};

struct DevFoldin {
    int32_t sweeps, burn_in, group;
    uint32_t key0, key1;
    double A;
    const FoldSlot *slots;  // [max_slots] control, written by the host
    int32_t *kept;          // [2*max_slots] kept, dropped: written by the device
    int32_t *prog;          // [2*max_slots] sweeps done, next token of the current sweep: device-written
    int32_t *words;         // arena [arena_tokens]
    int32_t *pos;           // arena: kept positions
    uint16_t *z;            // arena
    uint32_t *acc;          // [max_slots*K]
    float *theta;           // [max_slots*K]
    double *ll;             // [max_slots]
    int64_t *fin;           // [max_slots] the step that finished the request
                            // (written after theta and ll; 0 until then)
    int64_t step_no;        // this launch's step number (from 1)
};

hipError_t launch_foldin_step(const DevModel &m, const DevFoldin &f, const int32_t *active, int32_t n_active,
                              hipStream_t s);

// held-out log-likelihood of new documents (left-to-right estimate): the
// region of document d's particle r in kw, z and Zs starts at
// doc_off[d] * R + r * N_d (N_d = the document's length)
struct DevHeldout {
    int64_t D;
    int32_t R, group;
    uint32_t key0, key1;
    double A;                  // sum_k alpha_k
    const int64_t *doc_off;    // [D+1]
    const int32_t *words;      // [N]
    const uint32_t *req;       // [D] request ids (keys of the random numbers)
    const int32_t *order;      // [D] documents by decreasing length (longest chains start first)
    int32_t *kw;               // [R*N] each particle's kept words
    uint16_t *z;               // [R*N] each particle's topics
    double *Zs;                // [R*N] Z_n of each particle and step
    int32_t *kept;             // [D]
    double *ll;                // [D]
};

hipError_t launch_heldout(const DevModel &m, const DevHeldout &h, hipStream_t s);

}  // namespace pulda
