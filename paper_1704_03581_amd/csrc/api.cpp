// C ABI of libpulda.so (declared in include/pulda.h).
//
// Host side of the sampler: argument checks, the workspace layout, the
// Poisson alias tables of Section 3.4 (built once on the host), the z-step
// schedule (documents ordered by length, split into length buckets and work
// items), graph capture of a sweep, and the fold-in server's slot and arena
// bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pulda.h"
#include "internal.h"

using namespace pulda;

namespace {

thread_local std::string g_error;

pulda_status fail(pulda_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(PULDA_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t ALIGN = 256;
int64_t align_up(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Walker alias table by Vose's method: scaled probabilities p_j = (w_j n) / W
// (W the ascending sum), work lists of small (p < 1) and large entries in
// ascending order, first-in first-out; entries never paired keep
// probability 1 (threshold 0xFFFFFFFF, alias = self).
void alias_table(const std::vector<double> &w, std::vector<uint32_t> &thr, std::vector<int32_t> &alias)
{
    const int32_t n = (int32_t)w.size();
    double W = 0.0;
    for (double x : w) W += x;
    std::vector<double> p(n);
    std::vector<int32_t> work_small, work_large;
    work_small.reserve(2 * n);
    thr.assign(n, 0xFFFFFFFFu);
    alias.resize(n);
    for (int32_t j = 0; j < n; ++j) {
        p[j] = (w[j] * (double)n) / W;
        alias[j] = j;
        (p[j] < 1.0 ? work_small : work_large).push_back(j);
    }
    size_t si = 0, li = 0;
    while (si < work_small.size() && li < work_large.size()) {
        const int32_t s = work_small[si++];
        const int32_t g = work_large[li];
        thr[s] = (uint32_t)std::floor(p[s] * 4294967296.0);
        alias[s] = g;
        p[g] = (p[g] + p[s]) - 1.0;
        if (p[g] < 1.0) {
            ++li;
            work_small.push_back(g);
        }
    }
}

// Pois(beta + l), l = 1..L, on x = 0..X_l, X_l = ceil(lam + 10 sqrt(lam) + 10)
void poisson_tables(double beta, int32_t L, std::vector<int32_t> &off, std::vector<uint64_t> &packed)
{
    off.assign(L + 2, 0);
    packed.clear();
    for (int32_t l = 1; l <= L; ++l) {
        const double lam = beta + (double)l;
        const int32_t n = (int32_t)std::ceil(lam + 10.0 * std::sqrt(lam) + 10.0) + 1;
        std::vector<double> pmf(n);
        for (int32_t x = 0; x < n; ++x) pmf[x] = std::exp((double)x * std::log(lam) - lam - std::lgamma((double)x + 1.0));
        std::vector<uint32_t> thr;
        std::vector<int32_t> alias;
        alias_table(pmf, thr, alias);
        off[l] = (int32_t)packed.size();
        for (int32_t x = 0; x < n; ++x) packed.push_back((uint64_t)thr[x] | ((uint64_t)(uint32_t)alias[x] << 32));
    }
    off[L + 1] = (int32_t)packed.size();
}

// zero-truncated Pois(beta): T_x = floor(2^32 P(X <= x | X >= 1)), x = 1..,
// at least 5 entries, up to the first that saturates (the mass above it is
// below the 2^-32 resolution of the uniform that reads the table); appended
// to T, returns the count
constexpr int ZTP_CAP = 64;
constexpr double BETA_MAX = 16.0;   // rates whose tables saturate within ZTP_CAP

int32_t ztp_thresholds(double beta, std::vector<uint32_t> &T)
{
    const double norm = -std::expm1(-beta);
    double cdf = 0.0, term = std::exp(-beta);
    int32_t n = 0;
    for (int x = 1; x <= ZTP_CAP; ++x) {
        term = term * beta / (double)x;
        cdf += term;
        const double t = std::floor((cdf / norm) * 4294967296.0);
        T.push_back(t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t);
        ++n;
        if (x >= 5 && T.back() == 0xFFFFFFFFu) break;
    }
    return n;
}

struct Layout {
    int64_t total = 0;
    int64_t take(int64_t bytes)
    {
        const int64_t at = total;
        total = align_up(total + (bytes > 0 ? bytes : 1));
        return at;
    }
};

}  // namespace

struct pulda_plan {
    // model
    int32_t K = 0, V = 0, L = 100;
    double beta = 0.01, A = 0.0;
    uint64_t seed = 0;
    std::vector<double> alpha;
    int64_t D = 0, N = 0;
    // workspace
    uint8_t *ws = nullptr;
    int64_t ws_need = 0;
    struct {
        int64_t z, n, gam, phid, g16, Rd, gamd, Sd, dpart, phimax, wrec, hot, hot_word, beta_v, ztp, ztp_off, ckg, colcnt, colptr, ctopic, cphi, calias, sigma_a, S, nk, alpha, pois, pois_off,
            doc_order, items, queue, stats, ll_part, ll_out, ll_hist, tptr, err, scratch, cnt_a, ptr_a, cnt_b,
            ptr_b, zsave, lg_beta, lg_alpha, lg_A, ll_doc;
    } off;
    int64_t cap = 0, items_cap = 0, hist_cap = 4096;
    int32_t ks16 = 0;                 // row stride of the 16-bit draw table
    int32_t n_part_words = 1024, n_part_docs = 1024;
    std::vector<int32_t> pois_off_h;
    std::vector<uint64_t> pois_h;
    std::vector<double> lg_beta_h, lg_alpha_h, lg_A_h;  // log-joint term tables
    bool symmetric_alpha = true;
    std::vector<double> beta_vh;      // per-word priors (empty: the symmetric beta)
    std::vector<uint32_t> ztp_h;      // zero-truncated thresholds: one row, or one per word
    std::vector<int32_t> ztp_off_h;   // [V+1] row offsets for per-word priors
    int32_t ztp_n = 0;
    double beta_sum = 0.0;
    // device views
    DevModel m{};
    DevCorpus c{};
    WorkItem *items = nullptr;
    int32_t *queue = nullptr;
    unsigned long long *stats = nullptr;
    double *ll_part = nullptr, *ll_out = nullptr, *ll_hist = nullptr, *ll_doc = nullptr;
    uint32_t *tptr = nullptr, *hist_idx = nullptr;
    int32_t *err = nullptr;
    int64_t *cnt_a = nullptr, *ptr_a = nullptr, *cnt_b = nullptr, *ptr_b = nullptr;
    uint16_t *zsave = nullptr;
    // schedule
    std::vector<int32_t> len_sorted;  // lengths in doc_order
    std::vector<int32_t> min_len{1024, 256, 64, 0}, group{64, 64, 32, 16}, dpi{1, 2, 8, 32}, side{1, 1, 1, 1};
    int32_t n_items = 0;
    // work-item classes: (group size, count width) = (64, 16-bit), (32, 16),
    // (32, 8), (16, 16), (16, 8); 8-bit counts serve documents under 256 tokens
    static constexpr int NCLS = 7;
    static_assert(NCLS <= Z_QUEUES, "one work queue per class");
    int32_t cls_first[NCLS] = {}, cls_count[NCLS] = {};
    int32_t n_cu = 0;                 // compute units of the device
    // internal streams: the three group-size kernels of a z-step run
    // concurrently, forked from and joined back to the caller's stream
    hipStream_t aux[NCLS] = {};
    hipEvent_t fork_ev = nullptr, join_ev[NCLS] = {};
    // state
    bool bound = false, uploaded = false, have_z = false, have_phi = false;
    // graph replay
    bool graph_on = false;
    bool fused_ll = true;  // document terms of the log joint inside the z-step
    int32_t phi_method = PULDA_PHI_POLYA_URN;  // Phi-step of pulda_phi_step and pulda_sweep
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the sweep is captured on
    // phase timing (hipEvents on the caller's stream around each phase)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<size_t, size_t>> ev_phi, ev_z, ev_ll;
};

struct pulda_foldin {
    const pulda_plan *model = nullptr;
    pulda_foldin_desc desc{};
    int64_t ws_need = 0;
    struct {
        int64_t slots, kept, prog, words, pos, z, acc, theta, ll, fin, active;
    } off;
    uint8_t *ws = nullptr;
    DevFoldin f{};
    int32_t *active_dev = nullptr;
    FoldSlot *slots_dev = nullptr;
    // host bookkeeping
    std::vector<FoldSlot> slots;      // control mirror
    std::vector<int32_t> resident;    // 1 if the slot holds a request
    std::vector<int32_t> finished;    // 1 if its last sweep is known done (not yet collected)
    std::vector<int64_t> first_step;  // the step that took the occupant first (-1: none yet)
    std::vector<std::pair<int32_t, int32_t>> free_blocks;  // arena [off, len), by offset
    int32_t free_tokens = 0;
    int64_t n_steps = 0;              // steps launched
    // behind each step launch, an event (by step parity), and the stream on
    // which pulda_foldin_poll_previous reads results while the latest step
    // still runs
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    hipStream_t cstream = nullptr;
    // pinned host staging for the host-to-device copies, so that a copy
    // never reads caller or library memory after the call returns:
    // stage_words mirrors the arena (a region is rewritten only after its
    // request was polled, which waits for a step that ran after the region's
    // copy), and the slot table
    // and active list alternate between two buffers, each reused only after
    // the event recorded behind its previous copy
    int32_t *stage_words = nullptr;
    uint8_t *stage_ctl[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_cur = 0;
    ~pulda_foldin()
    {
        if (stage_words) (void)hipHostFree(stage_words);
        for (int b = 0; b < 2; ++b) {
            if (stage_ctl[b]) (void)hipHostFree(stage_ctl[b]);
            if (stage_ev[b]) (void)hipEventDestroy(stage_ev[b]);
            if (step_ev[b]) (void)hipEventDestroy(step_ev[b]);
        }
        if (cstream) (void)hipStreamDestroy(cstream);
    }
};

extern "C" {

const char *pulda_last_error(void) { return g_error.c_str(); }
const char *pulda_version(void) { return "pulda 0.1 (gfx950)"; }

pulda_status pulda_plan_create(const pulda_model_desc *desc, int64_t D, int64_t N, pulda_plan **out)
{
    if (!desc || !out) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (desc->K < 1 || desc->K > 4096) return fail(PULDA_ERR_INVALID_ARG, "K=%d outside 1..4096", desc->K);
    if (desc->V < 1) return fail(PULDA_ERR_INVALID_ARG, "V=%d must be >= 1", desc->V);
    // the kernels address the V x K tables (4-byte cells) with 32-bit byte
    // offsets
    if ((int64_t)desc->V * ((desc->K + 63) / 64 * 64) >= (1ll << 30))
        return fail(PULDA_ERR_INVALID_ARG, "V * (K rounded up to 64) must be < 2^30");
    if (!desc->beta_v && !(desc->beta > 0.0 && desc->beta <= BETA_MAX))
        return fail(PULDA_ERR_INVALID_ARG, "beta must be in (0, %g]", BETA_MAX);
    if (desc->beta_v)
        for (int32_t v = 0; v < desc->V; ++v)
            if (!(desc->beta_v[v] > 0.0 && desc->beta_v[v] <= BETA_MAX))
                return fail(PULDA_ERR_INVALID_ARG, "beta_v[%d] must be in (0, %g]", v, BETA_MAX);
    if (desc->L < 1 || desc->L > 1000) return fail(PULDA_ERR_INVALID_ARG, "L=%d outside 1..1000", desc->L);
    if (D < 0 || N < 0 || N >= (1ll << 40) || D >= (1ll << 31))
        return fail(PULDA_ERR_INVALID_ARG, "bad corpus size D=%lld N=%lld", (long long)D, (long long)N);
    std::vector<double> alpha(desc->K);
    for (int32_t k = 0; k < desc->K; ++k) {
        alpha[k] = desc->alpha_k ? desc->alpha_k[k] : desc->alpha;
        if (!(alpha[k] > 0.0) || !std::isfinite(alpha[k])) return fail(PULDA_ERR_INVALID_ARG, "alpha must be > 0");
    }
    pulda_plan *p = new pulda_plan();
    p->K = desc->K;
    p->V = desc->V;
    p->L = desc->L;
    p->beta = desc->beta_v ? 1.0 : desc->beta;   // (unused with per-word priors)
    if (desc->beta_v) p->beta_vh.assign(desc->beta_v, desc->beta_v + desc->V);
    p->seed = desc->seed;
    p->alpha = alpha;
    p->A = 0.0;
    for (double a : alpha) p->A += a;
    p->D = D;
    p->N = N;
    // per-word priors: tables of the integer rates l, and every cell's
    // Pois(beta_v) part from the prior marks
    poisson_tables(p->beta_vh.empty() ? p->beta : 0.0, p->L, p->pois_off_h, p->pois_h);
    if (p->beta_vh.empty()) {
        p->ztp_n = ztp_thresholds(p->beta, p->ztp_h);
        p->beta_sum = (double)p->V * p->beta;
    } else {
        p->ztp_off_h.assign(p->V + 1, 0);
        for (int32_t v = 0; v < p->V; ++v) {
            ztp_thresholds(p->beta_vh[v], p->ztp_h);
            p->ztp_off_h[v + 1] = (int32_t)p->ztp_h.size();
            p->beta_sum += p->beta_vh[v];
        }
    }
    // log-joint terms of small integer counts, evaluated once
    for (double a : alpha) p->symmetric_alpha = p->symmetric_alpha && a == alpha[0];
    p->lg_beta_h.resize(LG_TABLE);
    p->lg_alpha_h.resize(LG_TABLE);
    p->lg_A_h.resize(LG_TABLE);
    const double lgb = std::lgamma(p->beta), lga = std::lgamma(alpha[0]), lgA = std::lgamma(p->A);
    for (int32_t x = 0; x < LG_TABLE; ++x) {
        p->lg_beta_h[x] = std::lgamma((double)x + p->beta) - lgb;
        p->lg_alpha_h[x] = std::lgamma((double)x + alpha[0]) - lga;
        p->lg_A_h[x] = lgA - std::lgamma((double)x + p->A);
    }

    const int64_t VK = (int64_t)p->V * p->K;
    p->cap = VK;
    p->items_cap = D + 64;
    Layout L;
    p->off.z = L.take(N * 2);
    p->off.n = L.take(VK * 4);
    p->off.gam = L.take(VK * 4);
    p->off.phid = L.take(VK * 4);
    p->ks16 = (p->K + 63) / 64 * 64;
    p->off.g16 = L.take((int64_t)p->V * p->ks16 * 2);
    p->off.Rd = L.take((int64_t)p->K * 8);
    p->off.gamd = L.take(VK * 8);
    p->off.Sd = L.take((int64_t)p->K * 8);
    p->off.dpart = L.take(((int64_t)p->V + ROWSUM_COLS - 1) / ROWSUM_COLS * p->K * 8);
    p->off.colcnt = L.take((int64_t)p->V * 4);
    p->off.colptr = L.take(((int64_t)p->V + 1) * 4);
    p->off.ctopic = L.take(p->cap * 2);
    p->off.cphi = L.take(p->cap * 4);
    p->off.ckg = L.take(p->cap * 4);
    p->off.calias = L.take(p->cap * 8);
    p->off.sigma_a = L.take((int64_t)p->V * 8);
    p->off.beta_v = L.take(p->beta_vh.empty() ? 8 : (int64_t)p->V * 8);
    p->off.ztp = L.take((int64_t)p->ztp_h.size() * 4);
    p->off.ztp_off = L.take(((int64_t)p->V + 1) * 4);
    p->off.phimax = L.take((int64_t)p->V * 4);
    p->off.hot = L.take((int64_t)p->V * 4);
    p->off.hot_word = L.take((int64_t)HOT_MAX * 4);
    p->off.wrec = L.take((int64_t)p->V * 16);
    p->off.S = L.take((int64_t)p->K * 8);
    p->off.nk = L.take((int64_t)p->K * 8);
    p->off.alpha = L.take((int64_t)p->K * 8);
    p->off.pois = L.take((int64_t)p->pois_h.size() * 8);
    p->off.pois_off = L.take((int64_t)p->pois_off_h.size() * 4);
    p->off.doc_order = L.take(D * 4);
    p->off.items = L.take(p->items_cap * (int64_t)sizeof(WorkItem));
    p->off.queue = L.take(Z_QUEUES * 4);
    p->off.stats = L.take(ST_COUNT * 8);
    p->off.ll_part = L.take((int64_t)(p->n_part_words + p->n_part_docs) * 8);
    p->off.ll_out = L.take(8);
    p->off.ll_hist = L.take(p->hist_cap * 8);
    p->off.tptr = L.take(16);
    p->off.err = L.take(16);
    p->off.scratch = L.take((((int64_t)p->V + 1023) / 1024 + (D + 1023) / 1024 + 8) * 8);
    p->off.cnt_a = L.take(((int64_t)p->V + 2) * 8);
    p->off.ptr_a = L.take(((int64_t)p->V + 2) * 8);
    p->off.cnt_b = L.take((D + 2) * 8);
    p->off.ptr_b = L.take((D + 2) * 8);
    p->off.zsave = L.take(N * 2);
    p->off.lg_beta = L.take((int64_t)LG_TABLE * 8);
    p->off.lg_alpha = L.take((int64_t)LG_TABLE * 8);
    p->off.lg_A = L.take((int64_t)LG_TABLE * 8);
    p->off.ll_doc = L.take(D * 8);
    p->ws_need = L.total;
    *out = p;
    return PULDA_OK;
}

pulda_status pulda_plan_workspace_bytes(const pulda_plan *plan, int64_t *bytes)
{
    if (!plan || !bytes) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    *bytes = plan->ws_need;
    return PULDA_OK;
}

pulda_status pulda_plan_bind(pulda_plan *p, void *workspace_dev, int64_t bytes)
{
    if (!p || !workspace_dev) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if ((uintptr_t)workspace_dev % ALIGN) return fail(PULDA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < p->ws_need)
        return fail(PULDA_ERR_NO_MEMORY, "workspace of %lld bytes, need %lld", (long long)bytes, (long long)p->ws_need);
    uint8_t *w = (uint8_t *)workspace_dev;
    p->ws = w;
    DevModel &m = p->m;
    m.K = p->K;
    m.V = p->V;
    m.L = p->L;
    m.beta = p->beta;
    m.key0 = (uint32_t)p->seed;
    m.key1 = (uint32_t)(p->seed >> 32);
    m.alpha = (const double *)(w + p->off.alpha);
    m.n = (int32_t *)(w + p->off.n);
    m.nk = (unsigned long long *)(w + p->off.nk);
    m.gam = (int32_t *)(w + p->off.gam);
    m.S = (unsigned long long *)(w + p->off.S);
    m.phid = (float *)(w + p->off.phid);
    m.g16 = (uint16_t *)(w + p->off.g16);
    m.ks16 = p->ks16;
    m.Rd = (double *)(w + p->off.Rd);
    m.gamd = (double *)(w + p->off.gamd);
    m.Sd = (double *)(w + p->off.Sd);
    m.dpart = (double *)(w + p->off.dpart);
    m.phi_method = 0;
    m.ckg = (uint32_t *)(w + p->off.ckg);
    m.colcnt = (int32_t *)(w + p->off.colcnt);
    m.colptr = (int32_t *)(w + p->off.colptr);
    m.ctopic = (uint16_t *)(w + p->off.ctopic);
    m.cphi = (float *)(w + p->off.cphi);
    m.calias = (uint64_t *)(w + p->off.calias);
    m.sigma_a = (double *)(w + p->off.sigma_a);
    m.phimax = (float *)(w + p->off.phimax);
    m.hot = (int32_t *)(w + p->off.hot);
    m.hot_word = (int32_t *)(w + p->off.hot_word);
    m.n_hot = 0;
    m.wrec = (uint4 *)(w + p->off.wrec);
    m.pois = (const uint64_t *)(w + p->off.pois);
    m.pois_off = (const int32_t *)(w + p->off.pois_off);
    m.beta_v = p->beta_vh.empty() ? nullptr : (const double *)(w + p->off.beta_v);
    m.ztp_tab = (const uint32_t *)(w + p->off.ztp);
    m.ztp_off = p->beta_vh.empty() ? nullptr : (const int32_t *)(w + p->off.ztp_off);
    m.ztp_n = p->ztp_n;
    m.beta_sum = p->beta_sum;
    m.lg_beta = (const double *)(w + p->off.lg_beta);
    m.lg_alpha = p->symmetric_alpha ? (const double *)(w + p->off.lg_alpha) : nullptr;
    m.lg_A = (const double *)(w + p->off.lg_A);
    p->tptr = (uint32_t *)(w + p->off.tptr);
    p->hist_idx = p->tptr + 1;
    m.tptr = p->tptr;
    m.scratch = (long long *)(w + p->off.scratch);
    p->c.D = p->D;
    p->c.N = p->N;
    p->c.z = (uint16_t *)(w + p->off.z);
    p->c.doc_order = (const int32_t *)(w + p->off.doc_order);
    p->items = (WorkItem *)(w + p->off.items);
    p->queue = (int32_t *)(w + p->off.queue);
    p->stats = (unsigned long long *)(w + p->off.stats);
    p->ll_part = (double *)(w + p->off.ll_part);
    p->ll_out = (double *)(w + p->off.ll_out);
    p->ll_hist = (double *)(w + p->off.ll_hist);
    p->err = (int32_t *)(w + p->off.err);
    p->cnt_a = (int64_t *)(w + p->off.cnt_a);
    p->ptr_a = (int64_t *)(w + p->off.ptr_a);
    p->cnt_b = (int64_t *)(w + p->off.cnt_b);
    p->ptr_b = (int64_t *)(w + p->off.ptr_b);
    p->zsave = (uint16_t *)(w + p->off.zsave);
    p->ll_doc = (double *)(w + p->off.ll_doc);
    // constant tables (synchronous copies from host memory)
    HIP_TRY(hipMemcpy((void *)m.alpha, p->alpha.data(), p->K * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy((void *)m.pois, p->pois_h.data(), p->pois_h.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy((void *)m.pois_off, p->pois_off_h.data(), p->pois_off_h.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy((void *)m.ztp_tab, p->ztp_h.data(), p->ztp_h.size() * 4, hipMemcpyHostToDevice));
    if (m.beta_v) {
        HIP_TRY(hipMemcpy((void *)m.beta_v, p->beta_vh.data(), p->V * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy((void *)m.ztp_off, p->ztp_off_h.data(), (p->V + 1) * 4, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(w + p->off.lg_beta, p->lg_beta_h.data(), LG_TABLE * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w + p->off.lg_alpha, p->lg_alpha_h.data(), LG_TABLE * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w + p->off.lg_A, p->lg_A_h.data(), LG_TABLE * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(p->stats, 0, ST_COUNT * 8));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    p->n_cu = prop.multiProcessorCount;
    for (int c = 0; c < pulda_plan::NCLS; ++c) {
        if (!p->aux[c]) HIP_TRY(hipStreamCreateWithFlags(&p->aux[c], hipStreamNonBlocking));
        if (!p->join_ev[c]) HIP_TRY(hipEventCreateWithFlags(&p->join_ev[c], hipEventDisableTiming));
    }
    if (!p->fork_ev) HIP_TRY(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    p->bound = true;
    p->uploaded = p->have_z = p->have_phi = false;
    return PULDA_OK;
}

void pulda_plan_destroy(pulda_plan *p)
{
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (int c = 0; c < pulda_plan::NCLS; ++c) {
        if (p->aux[c]) (void)hipStreamDestroy(p->aux[c]);
        if (p->join_ev[c]) (void)hipEventDestroy(p->join_ev[c]);
    }
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
}

// record a pair of events around a phase when timing is on
static hipError_t phase_event(pulda_plan *p, hipStream_t s, size_t *idx)
{
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        p->ev_pool.push_back(e);
    }
    *idx = p->ev_used++;
    return hipEventRecord(p->ev_pool[*idx], s);
}

// a z-step class fits when one wave's count tables, topic lists and staged
// tokens take at most 32 KB of LDS (groups of 8 only for documents shorter
// than 256 tokens); one document per lane (group 1) takes documents shorter
// than 128 tokens (longest is the work item's longest document)
static bool class_fits(int32_t g, bool narrow, int32_t K, int32_t longest)
{
    // one document per lane: a list of at most 127 topics with 8-bit
    // counts (every list fits when K <= 127; a count stays below 256)
    if (g == 1) return longest < 128 || (K <= 127 && longest < 256);
    if (g == 8 && !narrow) return false;
    return z_layout(g, narrow, K).wave_bytes + 64 * 32 <= 32 * 1024;
}

static const int32_t kClassGroup[pulda_plan::NCLS] = {64, 32, 32, 16, 16, 8, 1};
static const bool kClassNarrow[pulda_plan::NCLS] = {false, false, true, false, true, true, true};

static int item_class(int32_t g, bool narrow)
{
    if (g == 64) return 0;
    if (g == 32) return narrow ? 2 : 1;
    if (g == 16) return narrow ? 4 : 3;
    if (g == 8) return 5;
    return 6;
}

static pulda_status build_items(pulda_plan *p)
{
    // items grouped by group size (64, 32, 16); within a group size in
    // decreasing document length (longest first)
    std::vector<WorkItem> cls[pulda_plan::NCLS];
    const int32_t nb = (int32_t)p->min_len.size();
    int64_t pos = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const int64_t start = pos;
        while (pos < p->D && p->len_sorted[pos] >= p->min_len[b]) ++pos;
        const int32_t per = p->dpi[b];
        for (int64_t s = start; s < pos; s += per) {
            WorkItem w;
            w.first = (int32_t)s;
            w.count = (int32_t)std::min<int64_t>(per, pos - s);
            w.side_ratio = p->side[b];
            // documents are in decreasing length: the first is the longest
            const bool narrow = p->len_sorted[s] < 256;
            // the bucket's group size, or the next larger one that fits
            int32_t g = p->group[b];
            if (g == 1 && !class_fits(1, narrow, p->K, p->len_sorted[s])) g = 16;
            while (g < 64 && !class_fits(g, narrow, p->K, p->len_sorted[s])) g *= 2;
            w.group = g;
            cls[item_class(w.group, narrow)].push_back(w);
        }
    }
    std::vector<WorkItem> items;
    for (int c = 0; c < pulda_plan::NCLS; ++c) {
        p->cls_first[c] = (int32_t)items.size();
        p->cls_count[c] = (int32_t)cls[c].size();
        items.insert(items.end(), cls[c].begin(), cls[c].end());
    }
    if ((int64_t)items.size() > p->items_cap) return fail(PULDA_ERR_INVALID_ARG, "schedule yields too many work items");
    p->n_items = (int32_t)items.size();
    if (!items.empty())
        HIP_TRY(hipMemcpy(p->items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    return PULDA_OK;
}

// The most frequent words (counted on a prefix of the corpus, at most 8M
// tokens): their count increments contend for few counters when K is small,
// so the z-step adds them up per block in LDS first.  As many words as
// HOT_BYTES of 32-bit counters hold at this K (none when that is under
// HOT_MIN).  Only where the increments are added changes, not the counts.
static hipError_t choose_hot_words(pulda_plan *p)
{
    p->m.n_hot = 0;
    const int32_t cap = HOT_BYTES / (4 * p->K);
    if (cap < HOT_MIN || p->N == 0) return hipSuccess;
    const int32_t n_hot = cap < p->V ? cap : p->V;
    const int64_t ns = p->N < (8ll << 20) ? p->N : (8ll << 20);
    std::vector<int32_t> w((size_t)ns);
    hipError_t e = hipMemcpy(w.data(), p->c.words, (size_t)ns * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    std::vector<int64_t> cnt((size_t)p->V, 0);
    for (int32_t v : w) cnt[(size_t)v]++;
    std::vector<int32_t> ids((size_t)p->V);
    for (int32_t v = 0; v < p->V; ++v) ids[(size_t)v] = v;
    std::partial_sort(ids.begin(), ids.begin() + n_hot, ids.end(), [&](int32_t a, int32_t b) {
        return cnt[(size_t)a] != cnt[(size_t)b] ? cnt[(size_t)a] > cnt[(size_t)b] : a < b;
    });
    std::vector<int32_t> hot((size_t)p->V, -1);
    for (int32_t h = 0; h < n_hot; ++h) hot[(size_t)ids[(size_t)h]] = h;
    e = hipMemcpy(p->m.hot, hot.data(), (size_t)p->V * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    e = hipMemcpy(p->m.hot_word, ids.data(), (size_t)n_hot * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    p->m.n_hot = n_hot;
    return hipSuccess;
}

pulda_status pulda_corpus_upload(pulda_plan *p, const int64_t *doc_off_dev, const int32_t *words_dev, void *stream)
{
    if (!p || (!doc_off_dev) || (!words_dev && p->N > 0)) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    p->c.doc_off = doc_off_dev;
    p->c.words = words_dev;
    HIP_TRY(launch_fill_u32((uint32_t *)p->err, 0u, 4, s));
    HIP_TRY(launch_validate(p->c, p->V, p->err, s));
    int32_t err[4];
    HIP_TRY(hipMemcpyAsync(err, p->err, sizeof(err), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err[0] || err[1] || err[2]) {
        p->uploaded = false;
        return fail(PULDA_ERR_CORPUS, "invalid corpus: %d bad offsets, %d word ids outside [0,%d), %d documents over "
                    "65535 tokens", err[0], err[1], p->V, err[2]);
    }
    // order documents by decreasing length (counting sort, stable in d)
    std::vector<int64_t> off(p->D + 1);
    HIP_TRY(hipMemcpy(off.data(), doc_off_dev, (p->D + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> hist(65537, 0);
    for (int64_t d = 0; d < p->D; ++d) hist[off[d + 1] - off[d]]++;
    std::vector<int64_t> start(65537, 0);
    int64_t run = 0;
    for (int32_t l = 65536; l >= 0; --l) {
        start[l] = run;
        run += hist[l];
    }
    std::vector<int32_t> order(p->D);
    p->len_sorted.assign(p->D, 0);
    for (int64_t d = 0; d < p->D; ++d) {
        const int64_t l = off[d + 1] - off[d];
        const int64_t at = start[l]++;
        order[at] = (int32_t)d;
        p->len_sorted[at] = (int32_t)l;
    }
    if (p->D) HIP_TRY(hipMemcpy((void *)p->c.doc_order, order.data(), p->D * 4, hipMemcpyHostToDevice));
    HIP_TRY(choose_hot_words(p));
    pulda_status st = build_items(p);
    if (st != PULDA_OK) return st;
    p->uploaded = true;
    p->have_z = false;
    return PULDA_OK;
}

pulda_status pulda_init(pulda_plan *p, const uint16_t *z0_dev, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->uploaded) return fail(PULDA_ERR_STATE, "no corpus uploaded");
    hipStream_t s = (hipStream_t)stream;
    if (z0_dev) {
        if (p->N) {
            HIP_TRY(hipMemcpyAsync(p->c.z, z0_dev, p->N * 2, hipMemcpyDeviceToDevice, s));
            HIP_TRY(launch_fill_u32((uint32_t *)p->err, 0u, 4, s));
            HIP_TRY(launch_check_u16_below(p->c.z, p->N, (uint32_t)p->K, p->err, s));
            int32_t bad = 0;
            HIP_TRY(hipMemcpyAsync(&bad, p->err, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (bad) {
                p->have_z = false;
                return fail(PULDA_ERR_INVALID_ARG, "%d topics in z are >= K=%d", bad, p->K);
            }
        }
    } else {
        HIP_TRY(launch_init_z(p->c, p->K, p->m.key0, p->m.key1, s));
    }
    HIP_TRY(launch_count_rebuild(p->c, p->m, s));
    p->have_z = true;
    return PULDA_OK;
}

pulda_status pulda_set_z(pulda_plan *p, const uint16_t *z_dev, void *stream)
{
    if (!p || (!z_dev && p->N > 0)) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    return pulda_init(p, z_dev, stream);
}

pulda_status pulda_get_z(const pulda_plan *p, uint16_t *z_dev, void *stream)
{
    if (!p || (!z_dev && p->N > 0)) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    if (p->N) HIP_TRY(hipMemcpyAsync(z_dev, p->c.z, p->N * 2, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return PULDA_OK;
}

pulda_status pulda_set_counts(pulda_plan *p, const int32_t *n_dev, void *stream)
{
    if (!p || !n_dev) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    HIP_TRY(hipMemcpyAsync(p->m.n, n_dev, (size_t)p->V * p->K * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    p->have_z = false;
    return PULDA_OK;
}

static pulda_status enqueue_phi(pulda_plan *p, hipStream_t s)
{
    size_t a = 0, b = 0;
    if (p->timing) HIP_TRY(phase_event(p, s, &a));
    p->m.phi_method = p->phi_method;
    if (p->phi_method == PULDA_PHI_DIRICHLET) HIP_TRY(launch_phi_step_dirichlet(p->m, p->stats, s));
    else HIP_TRY(launch_phi_step(p->m, p->stats, s));
    if (p->timing) {
        HIP_TRY(phase_event(p, s, &b));
        p->ev_phi.push_back({a, b});
    }
    return PULDA_OK;
}

// the z-step's launches (statistics into `stats`, or none)
static pulda_status enqueue_z_classes(pulda_plan *p, hipStream_t s, double *ll_doc, unsigned long long *stats)
{
    HIP_TRY(launch_z_prepare(p->m, p->queue, stats, s));
    int used = 0;
    for (int c = 0; c < pulda_plan::NCLS; ++c) used += p->cls_count[c] > 0;
    if (used <= 1) {
        for (int c = 0; c < pulda_plan::NCLS; ++c)
            if (p->cls_count[c])
                HIP_TRY(launch_z_class(p->c, p->m, kClassGroup[c], kClassNarrow[c], p->items + p->cls_first[c],
                                       p->cls_count[c], p->n_cu, p->queue + c, stats, ll_doc, s));
    } else {
        // classes run concurrently: long documents (large groups) next to
        // the bulk of short ones
        HIP_TRY(hipEventRecord(p->fork_ev, s));
        for (int c = 0; c < pulda_plan::NCLS; ++c) {
            if (!p->cls_count[c]) continue;
            HIP_TRY(hipStreamWaitEvent(p->aux[c], p->fork_ev, 0));
            HIP_TRY(launch_z_class(p->c, p->m, kClassGroup[c], kClassNarrow[c], p->items + p->cls_first[c],
                                   p->cls_count[c], p->n_cu, p->queue + c, stats, ll_doc, p->aux[c]));
            HIP_TRY(hipEventRecord(p->join_ev[c], p->aux[c]));
            HIP_TRY(hipStreamWaitEvent(s, p->join_ev[c], 0));
        }
    }
    return PULDA_OK;
}

static pulda_status enqueue_z(pulda_plan *p, hipStream_t s, double *ll_doc = nullptr)
{
    size_t ta = 0, tb = 0;
    if (p->timing) HIP_TRY(phase_event(p, s, &ta));
    pulda_status st = enqueue_z_classes(p, s, ll_doc, p->stats);
    if (st != PULDA_OK) return st;
    if (p->timing) {
        HIP_TRY(phase_event(p, s, &tb));
        p->ev_z.push_back({ta, tb});
    }
    return PULDA_OK;
}

static pulda_status enqueue_ll(pulda_plan *p, hipStream_t s, double *hist, const uint32_t *hist_idx,
                               const double *ll_doc = nullptr)
{
    size_t a = 0, b = 0;
    if (p->timing) HIP_TRY(phase_event(p, s, &a));
    HIP_TRY(launch_loglik(p->c, p->m, p->ll_part, p->n_part_words, p->n_part_docs, ll_doc, p->ll_out, hist,
                          hist_idx, s));
    if (p->timing) {
        HIP_TRY(phase_event(p, s, &b));
        p->ev_ll.push_back({a, b});
    }
    return PULDA_OK;
}

static bool counts_ready(const pulda_plan *p) { return p->have_z || !p->uploaded; }

pulda_status pulda_phi_step(pulda_plan *p, uint32_t t, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    if (t == 0) return fail(PULDA_ERR_INVALID_ARG, "sweeps are numbered from t = 1");
    (void)counts_ready;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_fill_u32(p->tptr, t, 1, s));
    pulda_status st = enqueue_phi(p, s);
    if (st == PULDA_OK) p->have_phi = true;
    return st;
}

pulda_status pulda_z_step(pulda_plan *p, uint32_t t, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    if (!p->have_phi) return fail(PULDA_ERR_STATE, "no Phi (call pulda_phi_step or pulda_set_phi)");
    if (t == 0) return fail(PULDA_ERR_INVALID_ARG, "sweeps are numbered from t = 1");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_fill_u32(p->tptr, t, 1, s));
    return enqueue_z(p, s);
}

static pulda_status enqueue_sweep_body(pulda_plan *p, hipStream_t s)
{
    pulda_status st = enqueue_phi(p, s);
    if (st != PULDA_OK) return st;
    // the z-step leaves each document's log-joint term behind (symmetric alpha)
    double *ll_doc = (p->symmetric_alpha && p->fused_ll) ? p->ll_doc : nullptr;
    st = enqueue_z(p, s, ll_doc);
    if (st != PULDA_OK) return st;
    st = enqueue_ll(p, s, p->ll_hist, p->hist_idx, ll_doc);
    if (st != PULDA_OK) return st;
    HIP_TRY(launch_advance(p->tptr, p->hist_idx, s));
    return PULDA_OK;
}

pulda_status pulda_sweep(pulda_plan *p, uint32_t t_first, int32_t n_sweeps, double *ll_host, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    if (t_first == 0 || n_sweeps < 0) return fail(PULDA_ERR_INVALID_ARG, "bad sweep range");
    hipStream_t s = (hipStream_t)stream;
    int32_t done = 0;
    while (done < n_sweeps) {
        const int32_t chunk = (int32_t)std::min<int64_t>(n_sweeps - done, p->hist_cap);
        HIP_TRY(launch_fill_u32(p->tptr, t_first + (uint32_t)done, 1, s));
        HIP_TRY(launch_fill_u32(p->hist_idx, 0u, 1, s));
        if (p->graph_on && !p->timing) {
            if (!p->gexec) {
                // capture one sweep on a private stream (the caller's stream
                // may be the legacy default stream, which cannot capture);
                // nothing runs during capture, the graph is then replayed on
                // the caller's stream
                if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
                hipGraph_t graph;
                HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
                pulda_status st = enqueue_sweep_body(p, p->cap_stream);
                hipError_t ec = hipStreamEndCapture(p->cap_stream, &graph);
                if (st != PULDA_OK) return st;
                if (ec != hipSuccess) return fail(PULDA_ERR_DEVICE, "graph capture: %s", hipGetErrorString(ec));
                ec = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ec != hipSuccess) return fail(PULDA_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(ec));
            }
            for (int32_t i = 0; i < chunk; ++i) HIP_TRY(hipGraphLaunch(p->gexec, s));
        } else {
            for (int32_t i = 0; i < chunk; ++i) {
                pulda_status st = enqueue_sweep_body(p, s);
                if (st != PULDA_OK) return st;
            }
        }
        if (ll_host) {
            HIP_TRY(hipMemcpyAsync(ll_host + done, p->ll_hist, chunk * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        done += chunk;
    }
    p->have_phi = true;
    return PULDA_OK;
}

pulda_status pulda_loglik(pulda_plan *p, double *ll_host, void *stream)
{
    if (!p || !ll_host) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    hipStream_t s = (hipStream_t)stream;
    pulda_status st = enqueue_ll(p, s, nullptr, nullptr, nullptr);
    if (st != PULDA_OK) return st;
    HIP_TRY(hipMemcpyAsync(ll_host, p->ll_out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PULDA_OK;
}

// ---------------------------------------------------------------------------
// counts and Phi export / import
// ---------------------------------------------------------------------------
static pulda_status count_sizes(pulda_plan *p, hipStream_t s, int64_t *nnz_n, int64_t *nnz_m)
{
    HIP_TRY(launch_n_colcount(p->m, p->cnt_a, s));
    HIP_TRY(launch_scan_i64(p->cnt_a, p->ptr_a, p->V, p->m.scratch, s));
    HIP_TRY(launch_counts_m(p->c, p->K, p->cnt_b, nullptr, nullptr, 0, s));
    HIP_TRY(launch_scan_i64(p->cnt_b, p->ptr_b, p->D, p->m.scratch + (p->V + 1023) / 1024 + 2, s));
    HIP_TRY(hipMemcpyAsync(nnz_n, p->ptr_a + p->V, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(nnz_m, p->ptr_b + p->D, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PULDA_OK;
}

pulda_status pulda_counts_sizes(pulda_plan *p, int64_t *nnz_n, int64_t *nnz_m, void *stream)
{
    if (!p || !nnz_n || !nnz_m) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    return count_sizes(p, (hipStream_t)stream, nnz_n, nnz_m);
}

pulda_status pulda_counts(pulda_plan *p, const pulda_counts_view *o, void *stream)
{
    if (!p || !o || !o->n_colptr_dev || !o->n_topic_dev || !o->n_count_dev || !o->m_rowptr_dev || !o->m_topic_dev ||
        !o->m_count_dev)
        return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_z) return fail(PULDA_ERR_STATE, "no state (call pulda_init)");
    hipStream_t s = (hipStream_t)stream;
    int64_t nn, nm;
    pulda_status st = count_sizes(p, s, &nn, &nm);
    if (st != PULDA_OK) return st;
    HIP_TRY(hipMemcpyAsync(o->n_colptr_dev, p->ptr_a, (p->V + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(o->m_rowptr_dev, p->ptr_b, (p->D + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_counts_csc(p->m, p->ptr_a, o->n_topic_dev, o->n_count_dev, nullptr, s));
    HIP_TRY(launch_counts_m(p->c, p->K, p->ptr_b, o->m_topic_dev, o->m_count_dev, 1, s));
    if (o->nk_dev) {
        HIP_TRY(launch_row_sums(p->m.n, p->V, p->K, p->m.nk, s));
        HIP_TRY(hipMemcpyAsync(o->nk_dev, p->m.nk, p->K * 8, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return PULDA_OK;
}

pulda_status pulda_get_counts_dense(pulda_plan *p, int32_t *n_dev, int64_t *nk_dev, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    if (n_dev) HIP_TRY(hipMemcpyAsync(n_dev, p->m.n, (size_t)p->V * p->K * 4, hipMemcpyDeviceToDevice, s));
    if (nk_dev) {
        HIP_TRY(launch_row_sums(p->m.n, p->V, p->K, p->m.nk, s));
        HIP_TRY(hipMemcpyAsync(nk_dev, p->m.nk, p->K * 8, hipMemcpyDeviceToDevice, s));
    }
    return PULDA_OK;
}

pulda_status pulda_phi_nnz(pulda_plan *p, int64_t *nnz, void *stream)
{
    if (!p || !nnz) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_phi) return fail(PULDA_ERR_STATE, "no Phi");
    hipStream_t s = (hipStream_t)stream;
    int32_t v;
    HIP_TRY(hipMemcpyAsync(&v, p->m.colptr + p->V, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *nnz = v;
    return PULDA_OK;
}

pulda_status pulda_get_phi(pulda_plan *p, const pulda_phi_view *o, void *stream)
{
    if (!p || !o || !o->colptr_dev || !o->topic_dev || !o->phi_dev || !o->alias_thr_dev || !o->alias_topic_dev ||
        !o->sigma_a_dev)
        return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_phi) return fail(PULDA_ERR_STATE, "no Phi");
    hipStream_t s = (hipStream_t)stream;
    int32_t *gam_e = o->gamma_dev;
    if (!gam_e) return fail(PULDA_ERR_INVALID_ARG, "gamma_dev is required for export");
    HIP_TRY(launch_export_phi(p->m, o->colptr_dev, o->topic_dev, gam_e, o->phi_dev, o->alias_thr_dev,
                              o->alias_topic_dev, s));
    HIP_TRY(hipMemcpyAsync(o->sigma_a_dev, p->m.sigma_a, p->V * 8, hipMemcpyDeviceToDevice, s));
    if (o->S_dev) HIP_TRY(hipMemcpyAsync(o->S_dev, p->m.S, p->K * 8, hipMemcpyDeviceToDevice, s));
    return PULDA_OK;
}

pulda_status pulda_set_phi(pulda_plan *p, const pulda_phi_view *in, void *stream)
{
    if (!p || !in || !in->colptr_dev || !in->topic_dev || !in->phi_dev || !in->alias_thr_dev ||
        !in->alias_topic_dev || !in->sigma_a_dev)
        return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    int64_t nnz;
    HIP_TRY(hipMemcpyAsync(&nnz, in->colptr_dev + p->V, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t first = 0;
    HIP_TRY(hipMemcpy(&first, in->colptr_dev, 8, hipMemcpyDeviceToHost));
    if (first != 0) return fail(PULDA_ERR_INVALID_ARG, "colptr[0] must be 0");
    if (nnz < 0 || nnz > p->cap) return fail(PULDA_ERR_INVALID_ARG, "Phi has %lld nonzeros, capacity %lld",
                                             (long long)nnz, (long long)p->cap);
    HIP_TRY(launch_fill_u32((uint32_t *)p->err, 0u, 4, s));
    HIP_TRY(launch_check_phi(in->colptr_dev, p->V, in->topic_dev, in->alias_topic_dev, (uint32_t)p->K, p->err, s));
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, p->err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return fail(PULDA_ERR_INVALID_ARG, "Phi has %d malformed columns or topics >= K", bad);
    HIP_TRY(launch_import_phi(p->m, in->colptr_dev, in->topic_dev, in->phi_dev, in->alias_thr_dev,
                              in->alias_topic_dev, s));
    HIP_TRY(hipMemcpyAsync(p->m.sigma_a, in->sigma_a_dev, p->V * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_word_records(p->m, s));
    // values without draws behind them: R_k = 0 keeps 0 * R_k finite for the
    // zero cells (every nonzero cell is read from phid)
    HIP_TRY(launch_fill_u64((unsigned long long *)p->m.Rd, 0ull, p->K, s));
    p->m.phi_method = PULDA_PHI_POLYA_URN;
    p->have_phi = true;
    return PULDA_OK;
}

// ---------------------------------------------------------------------------
// statistics, schedule, autotuning, graph
// ---------------------------------------------------------------------------
pulda_status pulda_stats(pulda_plan *p, pulda_sweep_stats *out, void *stream)
{
    if (!p || !out) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->bound) return fail(PULDA_ERR_STATE, "plan has no workspace bound");
    unsigned long long st[ST_COUNT];
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(st, p->stats, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->degenerate_tokens = (int64_t)st[ST_DEGENERATE];
    out->sum_J = (int64_t)st[ST_SUM_J];
    out->sum_J_b = (int64_t)st[ST_SUM_JB];
    out->fallback_draws = (int64_t)st[ST_FALLBACK];
    out->sum_A = (int64_t)st[ST_SUM_A];
    out->z_steps = (int64_t)st[ST_TOKENS];
    out->nnz_phi = (int64_t)st[ST_NNZ_PHI];
    out->empty_rows = (int64_t)st[ST_EMPTY_ROWS];
    auto total = [&](std::vector<std::pair<size_t, size_t>> &v, double *ms, int64_t *cnt) -> hipError_t {
        double t = 0.0;
        for (auto &pr : v) {
            float x = 0.0f;
            hipError_t e = hipEventElapsedTime(&x, p->ev_pool[pr.first], p->ev_pool[pr.second]);
            if (e != hipSuccess) return e;
            t += x;
        }
        *ms = t;
        *cnt = (int64_t)v.size();
        v.clear();
        return hipSuccess;
    };
    HIP_TRY(total(p->ev_phi, &out->ms_phi, &out->n_phi));
    HIP_TRY(total(p->ev_z, &out->ms_z, &out->n_z));
    HIP_TRY(total(p->ev_ll, &out->ms_ll, &out->n_ll));
    p->ev_used = 0;
    // z-step counters restart from zero
    HIP_TRY(launch_fill_u64(p->stats, 0ull, 3, s));
    HIP_TRY(launch_fill_u64(p->stats + ST_TOKENS, 0ull, 3, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PULDA_OK;
}

pulda_status pulda_set_schedule(pulda_plan *p, int32_t nb, const int32_t *min_len, const int32_t *group,
                                const int32_t *dpi, const int32_t *side_ratio)
{
    if (!p || nb < 1 || !min_len || !group || !dpi) return fail(PULDA_ERR_INVALID_ARG, "bad schedule");
    for (int32_t b = 0; b < nb; ++b) {
        if (group[b] != 1 && group[b] != 8 && group[b] != 16 && group[b] != 32 && group[b] != 64)
            return fail(PULDA_ERR_INVALID_ARG, "group size %d not in {1, 8, 16, 32, 64}", group[b]);
        if (dpi[b] < 1 || dpi[b] % (64 / group[b])) return fail(PULDA_ERR_INVALID_ARG, "docs per item %d", dpi[b]);
        if (b > 0 && min_len[b] >= min_len[b - 1]) return fail(PULDA_ERR_INVALID_ARG, "min_len must decrease");
        if (side_ratio && (side_ratio[b] < 1 || side_ratio[b] > 1024))
            return fail(PULDA_ERR_INVALID_ARG, "side ratio %d outside 1..1024", side_ratio[b]);
    }
    if (min_len[nb - 1] != 0) return fail(PULDA_ERR_INVALID_ARG, "last bucket must start at length 0");
    p->min_len.assign(min_len, min_len + nb);
    p->group.assign(group, group + nb);
    p->dpi.assign(dpi, dpi + nb);
    if (side_ratio) p->side.assign(side_ratio, side_ratio + nb);
    else p->side.assign(nb, 1);
    if (p->uploaded) return build_items(p);
    return PULDA_OK;
}

pulda_status pulda_get_schedule(const pulda_plan *p, int32_t cap, int32_t *nb, int32_t *min_len, int32_t *group,
                                int32_t *dpi, int32_t *side_ratio)
{
    if (!p || !nb) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    *nb = (int32_t)p->min_len.size();
    for (int32_t b = 0; b < *nb && b < cap; ++b) {
        if (min_len) min_len[b] = p->min_len[b];
        if (group) group[b] = p->group[b];
        if (dpi) dpi[b] = p->dpi[b];
        if (side_ratio) side_ratio[b] = p->side[b];
    }
    return PULDA_OK;
}

pulda_status pulda_autotune(pulda_plan *p, uint32_t t, int32_t reps, void *stream)
{
    if (!p || reps < 1 || t == 0) return fail(PULDA_ERR_INVALID_ARG, "bad argument");
    if (!p->have_z || !p->have_phi) return fail(PULDA_ERR_STATE, "autotune needs a state and a Phi");
    hipStream_t s = (hipStream_t)stream;
    if (p->N) HIP_TRY(hipMemcpyAsync(p->zsave, p->c.z, p->N * 2, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_fill_u32(p->tptr, t, 1, s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const std::vector<int32_t> keep_group = p->group, keep_dpi = p->dpi;
    const int32_t nb = (int32_t)p->min_len.size();
    std::vector<int32_t> best_g(keep_group), best_d(keep_dpi), best_r(p->side);
    std::vector<double> bucket_mean(nb, 0.0);   // mean document length (0: empty bucket)
    for (int32_t b = 0; b < nb; ++b) {
        // documents of bucket b
        int64_t lo = 0, hi = 0;
        {
            int64_t pos = 0;
            for (int32_t bb = 0; bb <= b; ++bb) {
                lo = pos;
                while (pos < p->D && p->len_sorted[pos] >= p->min_len[bb]) ++pos;
            }
            hi = pos;
        }
        if (hi == lo) continue;
        double mean_len = 0;
        for (int64_t i = lo; i < hi; ++i) mean_len += p->len_sorted[i];
        mean_len /= (double)(hi - lo);
        bucket_mean[b] = mean_len;
        float best_ms = 1e30f;
        const bool narrow = p->len_sorted[lo] < 256;
        for (int gsz : {64, 32, 16, 8, 1}) {
            if (!class_fits(gsz, narrow, p->K, p->len_sorted[lo])) continue;
            for (int ratio : {1, 4, 16}) {
                const int ng = 64 / gsz;
                int per = (int)std::max(1.0, std::round(4096.0 / std::max(1.0, mean_len) / ng)) * ng;
                std::vector<WorkItem> items;
                for (int64_t q = lo; q < hi; q += per)
                    items.push_back({(int32_t)q, (int32_t)std::min<int64_t>(per, hi - q), gsz, ratio});
                HIP_TRY(hipMemcpyAsync(p->items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                                       s));
                float total = 0;
                for (int r = 0; r <= reps; ++r) {
                    if (p->N) HIP_TRY(hipMemcpyAsync(p->c.z, p->zsave, p->N * 2, hipMemcpyDeviceToDevice, s));
                    HIP_TRY(hipEventRecord(e0, s));
                    HIP_TRY(launch_z_prepare(p->m, p->queue, nullptr, s));
                    HIP_TRY(launch_z_class(p->c, p->m, gsz, gsz < 64 && narrow, p->items,
                                           (int32_t)items.size(), p->n_cu, p->queue, nullptr, nullptr, s));
                    HIP_TRY(hipEventRecord(e1, s));
                    HIP_TRY(hipEventSynchronize(e1));
                    float ms;
                    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    if (r > 0) total += ms;  // first run warms up
                }
                if (total < best_ms) {
                    best_ms = total;
                    best_g[b] = gsz;
                    best_d[b] = per;
                    best_r[b] = ratio;
                }
            }
        }
    }
    p->group = best_g;
    p->dpi = best_d;
    p->side = best_r;
    pulda_status st = build_items(p);
    if (st != PULDA_OK) return st;
    // Then the whole z-step.  Each work-item class is a kernel of its own on
    // a forked stream, and a small class whose stream shares a hardware
    // queue with the caller's runs only after the others.  So each bucket is
    // also tried in every other bucket's group (and side ratio), and a change
    // is kept when the whole z-step, timed as the sweep launches it, is
    // faster.
    auto whole = [&](float *out) -> pulda_status {
        float total = 0;
        for (int r = 0; r <= reps; ++r) {
            if (p->N) HIP_TRY(hipMemcpyAsync(p->c.z, p->zsave, p->N * 2, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipEventRecord(e0, s));
            pulda_status q = enqueue_z_classes(p, s, nullptr, nullptr);
            if (q != PULDA_OK) return q;
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) total += ms;
        }
        *out = total;
        return PULDA_OK;
    };
    float best_all = 0;
    st = whole(&best_all);
    if (st != PULDA_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return st;
    }
    for (int32_t b = 0; b < nb; ++b) {
        if (bucket_mean[b] == 0) continue;
        for (int32_t b2 = 0; b2 < nb; ++b2) {
            if (b2 == b || bucket_mean[b2] == 0 || p->group[b2] == p->group[b]) continue;
            const int32_t g0 = p->group[b], d0 = p->dpi[b], r0 = p->side[b];
            const int32_t gsz = p->group[b2];
            const int ng = 64 / gsz;
            p->group[b] = gsz;
            p->dpi[b] = (int32_t)std::max(1.0, std::round(4096.0 / std::max(1.0, bucket_mean[b]) / ng)) * ng;
            p->side[b] = p->side[b2];
            float ms = 0;
            st = build_items(p);
            if (st == PULDA_OK) st = whole(&ms);
            if (st == PULDA_OK && ms < best_all) {
                best_all = ms;
            } else {
                p->group[b] = g0;
                p->dpi[b] = d0;
                p->side[b] = r0;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = build_items(p);
    if (st != PULDA_OK) return st;
    if (p->N) HIP_TRY(hipMemcpyAsync(p->c.z, p->zsave, p->N * 2, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_count_rebuild(p->c, p->m, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PULDA_OK;
}

pulda_status pulda_set_timing(pulda_plan *p, int32_t enable)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    p->timing = enable != 0;
    p->ev_phi.clear();
    p->ev_z.clear();
    p->ev_ll.clear();
    p->ev_used = 0;
    return PULDA_OK;
}

pulda_status pulda_set_fused_loglik(pulda_plan *p, int32_t enable)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    p->fused_ll = enable != 0;
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    return PULDA_OK;
}

pulda_status pulda_set_phi_method(pulda_plan *p, int32_t method)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (method != PULDA_PHI_POLYA_URN && method != PULDA_PHI_DIRICHLET)
        return fail(PULDA_ERR_INVALID_ARG, "unknown Phi-step method %d", method);
    p->phi_method = method;
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    return PULDA_OK;
}

pulda_status pulda_get_gamma_dense(pulda_plan *p, double *gamma_dev, double *S_dev, void *stream)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!p->have_phi || p->m.phi_method != PULDA_PHI_DIRICHLET)
        return fail(PULDA_ERR_STATE, "the last Phi-step was not a Dirichlet Phi-step");
    hipStream_t s = (hipStream_t)stream;
    if (gamma_dev)
        HIP_TRY(hipMemcpyAsync(gamma_dev, p->m.gamd, (size_t)p->V * p->K * 8, hipMemcpyDeviceToDevice, s));
    if (S_dev) HIP_TRY(hipMemcpyAsync(S_dev, p->m.Sd, (size_t)p->K * 8, hipMemcpyDeviceToDevice, s));
    return PULDA_OK;
}

pulda_status pulda_set_graph(pulda_plan *p, int32_t enable)
{
    if (!p) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    p->graph_on = enable != 0;
    if (!p->graph_on && p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    return PULDA_OK;
}

// ---------------------------------------------------------------------------
// fold-in server
// ---------------------------------------------------------------------------
pulda_status pulda_foldin_create(const pulda_plan *model, const pulda_foldin_desc *d, pulda_foldin **out)
{
    if (!model || !d || !out) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (!model->have_phi) return fail(PULDA_ERR_STATE, "the model has no Phi");
    if (d->sweeps < 1 || d->burn_in < 0 || d->burn_in >= d->sweeps) return fail(PULDA_ERR_INVALID_ARG, "bad sweeps");
    if (d->max_slots < 1 || d->arena_tokens < 1 || d->max_len < 1 || d->max_len > d->arena_tokens ||
        d->max_len > 65535)
        return fail(PULDA_ERR_INVALID_ARG, "bad capacity");
    if (d->group != 16 && d->group != 32 && d->group != 64) return fail(PULDA_ERR_INVALID_ARG, "bad group");
    pulda_foldin *f = new pulda_foldin();
    f->model = model;
    f->desc = *d;
    Layout L;
    const int64_t S = d->max_slots, T = d->arena_tokens, K = model->K;
    f->off.slots = L.take(S * (int64_t)sizeof(FoldSlot));
    f->off.kept = L.take(S * 8);
    f->off.prog = L.take(S * 8);
    f->off.words = L.take(T * 4);
    f->off.pos = L.take(T * 4);
    f->off.z = L.take(T * 2);
    f->off.acc = L.take(S * K * 4);
    f->off.theta = L.take(S * K * 4);
    f->off.ll = L.take(S * 8);
    f->off.fin = L.take(S * 8);
    f->off.active = L.take(S * 4);
    f->ws_need = L.total;
    f->slots.assign(S, FoldSlot{});
    f->resident.assign(S, 0);
    f->finished.assign(S, 0);
    f->first_step.assign(S, -1);
    f->free_blocks = {{0, (int32_t)T}};
    f->free_tokens = (int32_t)T;
    *out = f;
    return PULDA_OK;
}

pulda_status pulda_foldin_workspace_bytes(const pulda_foldin *f, int64_t *bytes)
{
    if (!f || !bytes) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    *bytes = f->ws_need;
    return PULDA_OK;
}

pulda_status pulda_foldin_bind(pulda_foldin *f, void *ws, int64_t bytes)
{
    if (!f || !ws) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if ((uintptr_t)ws % ALIGN) return fail(PULDA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < f->ws_need)
        return fail(PULDA_ERR_NO_MEMORY, "workspace of %lld bytes, need %lld", (long long)bytes, (long long)f->ws_need);
    if (!f->stage_words) {
        const size_t S = (size_t)f->desc.max_slots;
        if (hipHostMalloc((void **)&f->stage_words, (size_t)f->desc.arena_tokens * 4, hipHostMallocDefault) !=
            hipSuccess) {
            f->stage_words = nullptr;
            return fail(PULDA_ERR_NO_MEMORY, "pinned host staging of %d tokens", f->desc.arena_tokens);
        }
        for (int b = 0; b < 2; ++b) {
            if (hipHostMalloc((void **)&f->stage_ctl[b], S * (sizeof(FoldSlot) + 4), hipHostMallocDefault) !=
                hipSuccess) {
                f->stage_ctl[b] = nullptr;
                return fail(PULDA_ERR_NO_MEMORY, "pinned host staging of %zu slots", S);
            }
            HIP_TRY(hipEventCreateWithFlags(&f->stage_ev[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&f->step_ev[b], hipEventDisableTiming));
        }
        HIP_TRY(hipStreamCreateWithFlags(&f->cstream, hipStreamNonBlocking));
    }
    uint8_t *w = (uint8_t *)ws;
    f->ws = w;
    f->slots_dev = (FoldSlot *)(w + f->off.slots);
    f->active_dev = (int32_t *)(w + f->off.active);
    DevFoldin &F = f->f;
    F.sweeps = f->desc.sweeps;
    F.burn_in = f->desc.burn_in;
    F.group = f->desc.group;
    F.key0 = (uint32_t)f->desc.seed;
    F.key1 = (uint32_t)(f->desc.seed >> 32);
    F.A = f->model->A;
    F.slots = f->slots_dev;
    F.kept = (int32_t *)(w + f->off.kept);
    F.prog = (int32_t *)(w + f->off.prog);
    F.words = (int32_t *)(w + f->off.words);
    F.pos = (int32_t *)(w + f->off.pos);
    F.z = (uint16_t *)(w + f->off.z);
    F.acc = (uint32_t *)(w + f->off.acc);
    F.theta = (float *)(w + f->off.theta);
    F.ll = (double *)(w + f->off.ll);
    F.fin = (int64_t *)(w + f->off.fin);
    return PULDA_OK;
}

void pulda_foldin_destroy(pulda_foldin *f) { delete f; }

static bool arena_alloc(pulda_foldin *f, int32_t len, int32_t *at)
{
    const int32_t need = std::max(len, 1);
    for (size_t i = 0; i < f->free_blocks.size(); ++i) {
        auto &b = f->free_blocks[i];
        if (b.second >= need) {
            *at = b.first;
            b.first += need;
            b.second -= need;
            if (b.second == 0) f->free_blocks.erase(f->free_blocks.begin() + i);
            f->free_tokens -= need;
            return true;
        }
    }
    return false;
}

static void arena_free(pulda_foldin *f, int32_t at, int32_t len)
{
    const int32_t n = std::max(len, 1);
    auto &fb = f->free_blocks;
    auto it = std::lower_bound(fb.begin(), fb.end(), std::make_pair(at, 0));
    it = fb.insert(it, {at, n});
    f->free_tokens += n;
    size_t i = it - fb.begin();
    if (i + 1 < fb.size() && fb[i].first + fb[i].second == fb[i + 1].first) {
        fb[i].second += fb[i + 1].second;
        fb.erase(fb.begin() + i + 1);
    }
    if (i > 0 && fb[i - 1].first + fb[i - 1].second == fb[i].first) {
        fb[i - 1].second += fb[i].second;
        fb.erase(fb.begin() + i);
    }
}

pulda_status pulda_foldin_submit(pulda_foldin *f, uint32_t req, const int32_t *words, int32_t len, void *stream)
{
    if (!f || (len > 0 && !words)) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!f->ws) return fail(PULDA_ERR_STATE, "no workspace bound");
    if (len < 0 || len > f->desc.max_len)
        return fail(PULDA_ERR_INVALID_ARG, "request length %d outside 0..%d", len, f->desc.max_len);
    int32_t sid = -1;
    for (int32_t i = 0; i < f->desc.max_slots; ++i)
        if (!f->resident[i]) {
            sid = i;
            break;
        }
    if (sid < 0) return fail(PULDA_ERR_CAPACITY, "no free slot");
    int32_t at;
    if (!arena_alloc(f, len, &at)) return fail(PULDA_ERR_CAPACITY, "no arena space for %d tokens", len);
    hipStream_t s = (hipStream_t)stream;
    if (len > 0) {
        std::memcpy(f->stage_words + at, words, (size_t)len * 4);
        hipError_t e = hipMemcpyAsync(f->f.words + at, f->stage_words + at, (size_t)len * 4, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            arena_free(f, at, len);
            return fail(PULDA_ERR_DEVICE, "copy request: %s", hipGetErrorString(e));
        }
    }
    FoldSlot &sl = f->slots[sid];
    sl.arena_off = at;
    sl.len = len;
    sl.req = req;
    sl.fresh = 1;
    sl.budget = 0;
    f->resident[sid] = 1;
    f->finished[sid] = 0;
    f->first_step[sid] = -1;
    return PULDA_OK;
}

pulda_status pulda_foldin_step(pulda_foldin *f, int32_t draws, void *stream)
{
    if (!f || draws < 1) return fail(PULDA_ERR_INVALID_ARG, "bad argument");
    if (!f->ws) return fail(PULDA_ERR_STATE, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    const int b = f->stage_cur;
    if (f->stage_used[b]) HIP_TRY(hipEventSynchronize(f->stage_ev[b]));
    const int32_t S = f->desc.max_slots;
    FoldSlot *slots_pin = (FoldSlot *)f->stage_ctl[b];
    int32_t *active = (int32_t *)(f->stage_ctl[b] + (size_t)S * sizeof(FoldSlot));
    int32_t n_active = 0;
    const int64_t step_no = f->n_steps + 1;
    for (int32_t i = 0; i < S; ++i) {
        FoldSlot &sl = f->slots[i];
        if (f->resident[i] && !f->finished[i]) {
            sl.budget = draws;
            active[n_active++] = i;
            if (sl.fresh) f->first_step[i] = step_no;
        } else {
            sl.budget = 0;
        }
    }
    if (n_active == 0) return PULDA_OK;
    std::memcpy(slots_pin, f->slots.data(), (size_t)S * sizeof(FoldSlot));
    HIP_TRY(hipMemcpyAsync(f->slots_dev, slots_pin, (size_t)S * sizeof(FoldSlot), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(f->active_dev, active, (size_t)n_active * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(f->stage_ev[b], s));
    f->stage_used[b] = true;
    f->stage_cur = b ^ 1;
    f->f.step_no = step_no;
    HIP_TRY(launch_foldin_step(f->model->m, f->f, f->active_dev, n_active, s));
    f->n_steps = step_no;
    HIP_TRY(hipEventRecord(f->step_ev[step_no & 1], s));
    for (int32_t j = 0; j < n_active; ++j) {
        f->slots[active[j]].fresh = 0;
        f->slots[active[j]].budget = 0;
    }
    return PULDA_OK;
}

// the requests finished by step `limit` (every step up to it complete on
// stream s): their results, up to cap of them, and their slots freed
static pulda_status foldin_collect(pulda_foldin *f, int64_t limit, hipStream_t s, pulda_foldin_result *out,
                                   float *theta, int32_t cap, int32_t *n_done)
{
    const int32_t K = f->model->K, S = f->desc.max_slots;
    *n_done = 0;
    bool any = false;
    for (int32_t i = 0; i < S; ++i) any |= f->resident[i] && f->first_step[i] > 0 && f->first_step[i] <= limit;
    if (!any) return PULDA_OK;
    // a slot's fin is the step that wrote its theta and log-likelihood;
    // steps after `limit` may be running, so later values are not yet safe
    std::vector<int64_t> fin(S);
    std::vector<int32_t> kept(2 * S);
    std::vector<double> ll(S);
    HIP_TRY(hipMemcpyAsync(fin.data(), f->f.fin, fin.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(kept.data(), f->f.kept, kept.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ll.data(), f->f.ll, ll.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> done;
    for (int32_t i = 0; i < S; ++i) {
        if (!f->resident[i] || f->first_step[i] < 1 || f->first_step[i] > limit) continue;
        if (fin[i] < f->first_step[i] || fin[i] > limit) continue;
        f->finished[i] = 1;
        if ((int32_t)done.size() < cap) done.push_back(i);
    }
    if (done.empty()) return PULDA_OK;
    for (size_t j = 0; j < done.size(); ++j)
        HIP_TRY(hipMemcpyAsync(theta + j * K, f->f.theta + (int64_t)done[j] * K, K * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t j = 0; j < done.size(); ++j) {
        const int32_t i = done[j];
        out[j].request_id = f->slots[i].req;
        out[j].kept = kept[2 * i];
        out[j].dropped = kept[2 * i + 1];
        out[j].pad = 0;
        out[j].loglik = ll[i];
        f->resident[i] = 0;
        f->finished[i] = 0;
        f->first_step[i] = -1;
        arena_free(f, f->slots[i].arena_off, f->slots[i].len);
    }
    *n_done = (int32_t)done.size();
    return PULDA_OK;
}

pulda_status pulda_foldin_poll(pulda_foldin *f, pulda_foldin_result *out, float *theta, int32_t cap, int32_t *n_done,
                               void *stream)
{
    if (!f || !n_done || (cap > 0 && (!out || !theta))) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!f->ws) return fail(PULDA_ERR_STATE, "no workspace bound");
    // (the copies queue behind every step launched on the stream)
    return foldin_collect(f, f->n_steps, (hipStream_t)stream, out, theta, cap, n_done);
}

pulda_status pulda_foldin_poll_previous(pulda_foldin *f, pulda_foldin_result *out, float *theta, int32_t cap,
                                        int32_t *n_done)
{
    if (!f || !n_done || (cap > 0 && (!out || !theta))) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!f->ws) return fail(PULDA_ERR_STATE, "no workspace bound");
    *n_done = 0;
    const int64_t limit = f->n_steps - 1;
    if (limit < 1) return PULDA_OK;
    // the library's copy stream waits for step `limit` only; the latest step
    // keeps running (it skips the requests finished before it)
    HIP_TRY(hipStreamWaitEvent(f->cstream, f->step_ev[limit & 1], 0));
    return foldin_collect(f, limit, f->cstream, out, theta, cap, n_done);
}

pulda_status pulda_foldin_occupancy(const pulda_foldin *f, int32_t *resident, int32_t *free_slots,
                                    int32_t *free_tokens)
{
    if (!f) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    int32_t r = 0;
    for (int32_t x : f->resident) r += x;
    if (resident) *resident = r;
    if (free_slots) *free_slots = f->desc.max_slots - r;
    if (free_tokens) *free_tokens = f->free_tokens;
    return PULDA_OK;
}

pulda_status pulda_foldin_run_one(pulda_foldin *f, uint32_t req, const int32_t *words, int32_t len, float *theta,
                                  pulda_foldin_result *out, void *stream)
{
    if (!f || !theta || !out) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    int32_t r = 0;
    for (int32_t x : f->resident) r += x;
    if (r) return fail(PULDA_ERR_STATE, "the server holds %d requests", r);
    pulda_status st = pulda_foldin_submit(f, req, words, len, stream);
    if (st != PULDA_OK) return st;
    st = pulda_foldin_step(f, INT32_MAX, stream);
    if (st != PULDA_OK) return st;
    int32_t n = 0;
    st = pulda_foldin_poll(f, out, theta, 1, &n, stream);
    if (st != PULDA_OK) return st;
    if (n != 1) return fail(PULDA_ERR_DEVICE, "request did not finish");
    return PULDA_OK;
}

// ---------------------------------------------------------------------------
// Held-out log-likelihood (left-to-right estimate)
// ---------------------------------------------------------------------------
static int64_t heldout_bytes(int64_t D, int64_t N, int32_t R)
{
    Layout L;
    L.take(D * 4);
    L.take(N * R * 4);
    L.take(N * R * 2);
    L.take(N * R * 8);
    return L.total;
}

pulda_status pulda_heldout_workspace_bytes(const pulda_plan *model, int64_t D, int64_t N, int32_t particles,
                                           int64_t *bytes)
{
    if (!model || !bytes) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (D < 0 || N < 0 || particles < 1 || particles >= (1 << 24))
        return fail(PULDA_ERR_INVALID_ARG, "D=%lld, N=%lld, particles=%d", (long long)D, (long long)N, particles);
    *bytes = heldout_bytes(D, N, particles);
    return PULDA_OK;
}

}  // extern "C"

// The held-out estimate with its scratch at workspace_dev (workspace_bytes
// long, 256-byte aligned).  from_static: the scratch is the library's own
// per-device array (the message of a size error names its limit).
static pulda_status heldout_run(const pulda_plan *model, int64_t D, const int64_t *doc_off_dev,
                                const int32_t *words_dev, const uint32_t *req_dev, int32_t particles, int32_t group,
                                uint64_t seed, void *workspace_dev, int64_t workspace_bytes, double *ll_dev,
                                int32_t *kept_dev, double *Z_dev, void *stream, bool from_static)
{
    if (!model || !doc_off_dev || !req_dev || !ll_dev || !kept_dev || (D > 0 && !workspace_dev))
        return fail(PULDA_ERR_INVALID_ARG, "null argument");
    if (!model->have_phi) return fail(PULDA_ERR_STATE, "the model has no Phi");
    if (D < 0 || D >= (1ll << 31)) return fail(PULDA_ERR_INVALID_ARG, "D=%lld", (long long)D);
    if (particles < 1 || particles >= (1 << 24)) return fail(PULDA_ERR_INVALID_ARG, "particles=%d", particles);
    if (group != 16 && group != 32 && group != 64) return fail(PULDA_ERR_INVALID_ARG, "group %d", group);
    if ((uintptr_t)workspace_dev % ALIGN) return fail(PULDA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (D == 0) return PULDA_OK;
    hipStream_t s = (hipStream_t)stream;
    // the offsets are checked on the host before any launch
    std::vector<int64_t> off(D + 1);
    HIP_TRY(hipMemcpyAsync(off.data(), doc_off_dev, (D + 1) * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (off[0] != 0) return fail(PULDA_ERR_CORPUS, "doc_off[0] = %lld", (long long)off[0]);
    for (int64_t d = 0; d < D; ++d)
        if (off[d + 1] < off[d] || off[d + 1] - off[d] > 65535)
            return fail(PULDA_ERR_CORPUS, "document %lld: offsets %lld..%lld", (long long)d, (long long)off[d],
                        (long long)off[d + 1]);
    const int64_t N = off[D];
    if (N > 0 && !words_dev) return fail(PULDA_ERR_INVALID_ARG, "null words");
    if (N * particles >= (1ll << 40)) return fail(PULDA_ERR_INVALID_ARG, "N * particles too large");
    if (workspace_bytes < heldout_bytes(D, N, particles)) {
        if (from_static)
            return fail(PULDA_ERR_NO_MEMORY,
                        "%lld documents, %lld tokens and %d particles need %lld bytes of scratch; the library's "
                        "own scratch holds %lld (use pulda_heldout_loglik with a workspace)",
                        (long long)D, (long long)N, particles, (long long)heldout_bytes(D, N, particles),
                        (long long)workspace_bytes);
        return fail(PULDA_ERR_NO_MEMORY, "workspace of %lld bytes, need %lld", (long long)workspace_bytes,
                    (long long)heldout_bytes(D, N, particles));
    }
    // longest documents first: each particle is a chain of ~n^2/2 draws, so
    // the long ones set the call's time unless they start early
    std::vector<int32_t> order(D);
    for (int64_t d = 0; d < D; ++d) order[d] = (int32_t)d;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
    Layout L;
    uint8_t *w = (uint8_t *)workspace_dev;
    int32_t *order_dev = (int32_t *)(w + L.take(D * 4));
    HIP_TRY(hipMemcpyAsync(order_dev, order.data(), D * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host array ends with this call
    DevHeldout h{};
    h.D = D;
    h.R = particles;
    h.group = group;
    h.key0 = (uint32_t)seed;
    h.key1 = (uint32_t)(seed >> 32);
    h.A = model->A;
    h.doc_off = doc_off_dev;
    h.words = words_dev;
    h.req = req_dev;
    h.order = order_dev;
    h.kw = (int32_t *)(w + L.take(N * particles * 4));
    h.z = (uint16_t *)(w + L.take(N * particles * 2));
    const int64_t zs_off = L.take(N * particles * 8);
    h.Zs = Z_dev ? Z_dev : (double *)(w + zs_off);
    h.kept = kept_dev;
    h.ll = ll_dev;
    HIP_TRY(launch_heldout(model->m, h, s));
    return PULDA_OK;
}

// The scratch of pulda_heldout_loglik_noalloc: one array per GPU the library
// runs on, held until the process ends.  Host code never uses the array's
// name as an address: the device address of each GPU's copy is looked up
// once (hipGetSymbolAddress, with that device current) and kept per device.
static __device__ __align__(256) uint8_t scratch[PULDA_HELDOUT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_SCRATCH_DEVICES];
}  // namespace

static pulda_status scratch_of_current_device(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return fail(PULDA_ERR_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PULDA_ERR_DEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PULDA_OK;
}

extern "C" {

pulda_status pulda_heldout_loglik(const pulda_plan *model, int64_t D, const int64_t *doc_off_dev,
                                  const int32_t *words_dev, const uint32_t *req_dev, int32_t particles, int32_t group,
                                  uint64_t seed, void *workspace_dev, int64_t workspace_bytes, double *ll_dev,
                                  int32_t *kept_dev, double *Z_dev, void *stream)
{
    return heldout_run(model, D, doc_off_dev, words_dev, req_dev, particles, group, seed, workspace_dev,
                       workspace_bytes, ll_dev, kept_dev, Z_dev, stream, false);
}

pulda_status pulda_heldout_loglik_noalloc(const pulda_plan *model, int64_t D, const int64_t *doc_off_dev,
                                          const int32_t *words_dev, const uint32_t *req_dev, int32_t particles,
                                          int32_t group, uint64_t seed, double *ll_dev, int32_t *kept_dev,
                                          double *Z_dev, void *stream)
{
    if (!model) return fail(PULDA_ERR_INVALID_ARG, "null argument");
    void *ws = nullptr;
    const pulda_status st = scratch_of_current_device(&ws);
    if (st != PULDA_OK) return st;
    return heldout_run(model, D, doc_off_dev, words_dev, req_dev, particles, group, seed, ws,
                       PULDA_HELDOUT_NOALLOC_SCRATCH_BYTES, ll_dev, kept_dev, Z_dev, stream, true);
}

}  // extern "C"
