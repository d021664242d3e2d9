// HIP kernels of the Polya-urn partially collapsed LDA sampler for gfx950.
//
// Algorithm 2 of the paper (Section 3): every sweep draws each topic row
// phi_k ~ PPU(n_k + beta) (the Phi-step), then every token's topic from
// P(z_i = k) propto phi_{k,v(i)} (alpha_k + m^{-i}_{d,k}) (the z-step), and the
// counts n, m are rebuilt from z.  Section 3.4 gives the Poisson draws (alias
// tables for rates beta + l, l <= L; rounded Gaussian above), Section 3.5 the
// a/b split of the token conditional and the doubly sparse b-sum.
//
// Layouts in HBM (all word-major, so one word's column is contiguous):
//   n[v*K + k], gam[v*K + k], phid[v*K + k]    dense K x V tables
//   colptr[v] .. colptr[v+1]                    CSC of Phi's nonzeros by word,
//     ctopic (u16, ascending), cphi (f32), calias (u64: thr | topic << 32 |
//     alias topic << 48)
//   doc_off[d] .. doc_off[d+1]                  CSR tokens, words (i32), z (u16)
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace pulda {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long value, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

static int grid_for(int64_t n, int block, int cap = 65536)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    fill_u32_kernel<<<grid_for(count, 256, 16384), 256, 0, s>>>(p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    fill_u64_kernel<<<grid_for(count, 256, 16384), 256, 0, s>>>(p, value, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scans (three passes: block sums, scan of block sums, add-back)
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 1024;

template <typename Tin>
__global__ void scan_block_sums(const Tin *in, int64_t n, long long *bsum)
{
    __shared__ long long part[SCAN_BLOCK / 64];
    int64_t i = blockIdx.x * (int64_t)SCAN_BLOCK + threadIdx.x;
    long long x = i < n ? (long long)in[i] : 0;
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < SCAN_BLOCK / 64; ++w) t += part[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ void scan_sums_serial(long long *bsum, int64_t nb, long long *total)
{
    // one block: each thread scans a contiguous chunk, then chunk offsets are combined
    __shared__ long long chunk[1024];
    int64_t per = (nb + blockDim.x - 1) / blockDim.x;
    int64_t a = threadIdx.x * per, b = a + per < nb ? a + per : nb;
    long long t = 0;
    for (int64_t i = a; i < b; ++i) t += bsum[i];
    chunk[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int j = 0; j < (int)blockDim.x; ++j) {
            long long c = chunk[j];
            chunk[j] = run;
            run += c;
        }
        if (total) *total = run;
    }
    __syncthreads();
    long long run = chunk[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        long long c = bsum[i];
        bsum[i] = run;
        run += c;
    }
}

template <typename Tin, typename Tout>
__global__ void scan_apply(const Tin *in, int64_t n, const long long *boff, Tout *out)
{
    __shared__ long long wsum[SCAN_BLOCK / 64];
    int64_t i = blockIdx.x * (int64_t)SCAN_BLOCK + threadIdx.x;
    long long x = i < n ? (long long)in[i] : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        long long y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    long long before = boff[blockIdx.x];
    for (int j = 0; j < w; ++j) before += wsum[j];
    if (i < n) out[i] = (Tout)(before + incl - x);
    if (i == n - 1) out[n] = (Tout)(before + incl);
}

template <typename Tin, typename Tout>
static hipError_t scan_excl(const Tin *in, Tout *out, int64_t n, long long *scratch, long long *total,
                            hipStream_t s)
{
    // out has n + 1 entries; scratch holds ceil(n / SCAN_BLOCK) entries
    if (n <= 0) {
        scan_sums_serial<<<1, 64, 0, s>>>(scratch, 0, total);
        return hipGetLastError();
    }
    int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    scan_block_sums<Tin><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, scratch);
    scan_sums_serial<<<1, 1024, 0, s>>>(scratch, nb, total);
    scan_apply<Tin, Tout><<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, scratch, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// corpus validation: monotone offsets from 0 to N, word ids in [0, V),
// document lengths within the 16-bit per-document count range
// ---------------------------------------------------------------------------
__global__ void validate_kernel(const int64_t *doc_off, int64_t D, const int32_t *words, int64_t N, int32_t V,
                                int32_t *err)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < D; d += stride) {
        int64_t a = doc_off[d], b = doc_off[d + 1];
        if (b < a || a < 0 || b > N) atomicAdd(&err[0], 1);
        else if (b - a > 65535) atomicAdd(&err[2], 1);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (doc_off[0] != 0 || doc_off[D] != N) atomicAdd(&err[0], 1);
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += stride) {
        int32_t w = words[i];
        if (w < 0 || w >= V) atomicAdd(&err[1], 1);
    }
}

hipError_t launch_validate(const DevCorpus &c, int32_t V, int32_t *err, hipStream_t s)
{
    validate_kernel<<<grid_for(c.N > c.D ? c.N : c.D, 256, 8192), 256, 0, s>>>(c.doc_off, c.D, c.words, c.N, V, err);
    return hipGetLastError();
}

// caller-supplied state and Phi: every topic below K, columns well formed
__global__ void check_u16_below_kernel(const uint16_t *x, int64_t n, uint32_t limit, int32_t *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (x[i] >= limit) atomicAdd(err, 1);
}

hipError_t launch_check_u16_below(const uint16_t *x, int64_t n, uint32_t limit, int32_t *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    check_u16_below_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(x, n, limit, err);
    return hipGetLastError();
}

__global__ void check_phi_kernel(const int64_t *colptr, int32_t V, const uint16_t *topic, const uint16_t *alias_topic,
                                 uint32_t K, int32_t *err)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= V) return;
    const int lane = __lane_id();
    const int64_t a = colptr[v], b = colptr[v + 1];
    if (b < a || b - a > (int64_t)K) {
        if (lane == 0) atomicAdd(err, 1);
        return;
    }
    for (int64_t e = a + lane; e < b; e += 64) {
        const bool ok = topic[e] < K && alias_topic[e] < K && (e == a || topic[e - 1] < topic[e]);
        if (!ok) atomicAdd(err, 1);
    }
}

hipError_t launch_check_phi(const int64_t *colptr, int32_t V, const uint16_t *topic, const uint16_t *alias_topic,
                            uint32_t K, int32_t *err, hipStream_t s)
{
    check_phi_kernel<<<(V + 3) / 4, 256, 0, s>>>(colptr, V, topic, alias_topic, K, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initial state: z_i uniform on {0..K-1}
// ---------------------------------------------------------------------------
__global__ void init_z_kernel(uint16_t *z, int64_t N, int32_t K, uint32_t key0, uint32_t key1)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        r4 r = philox((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, TAG_INIT, key0, key1);
        z[i] = (uint16_t)scale32(r.x, (uint32_t)K);
    }
}

hipError_t launch_init_z(const DevCorpus &c, int32_t K, uint32_t key0, uint32_t key1, hipStream_t s)
{
    if (c.N == 0) return hipSuccess;
    init_z_kernel<<<grid_for(c.N, 256, 16384), 256, 0, s>>>(c.z, c.N, K, key0, key1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// count rebuild from z (Table 1): n[v*K + k] += 1 for every token
// ---------------------------------------------------------------------------
__global__ void count_tokens_kernel(const int32_t *words, const uint16_t *z, int64_t N, int32_t K, int32_t *n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&n[(int64_t)words[i] * K + z[i]], 1);
}

hipError_t launch_count_rebuild(const DevCorpus &c, const DevModel &m, hipStream_t s)
{
    hipError_t e = launch_fill_u32((uint32_t *)m.n, 0u, (int64_t)m.V * m.K, s);
    if (e != hipSuccess) return e;
    if (c.N == 0) return hipSuccess;
    count_tokens_kernel<<<grid_for(c.N, 256, 16384), 256, 0, s>>>(c.words, c.z, c.N, m.K, m.n);
    return hipGetLastError();
}

// column sums of a word-major V x K table: out[k] += sum_v dense[v*K + k]

__global__ void row_sums_kernel(const int32_t *dense, int32_t V, int32_t K, unsigned long long *out)
{
    const int32_t v0 = blockIdx.x * ROWSUM_COLS;
    const int32_t v1 = v0 + ROWSUM_COLS < V ? v0 + ROWSUM_COLS : V;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        unsigned long long t = 0;
        int32_t v = v0;
        // eight rows' loads in flight before they are added
        for (; v + 8 <= v1; v += 8) {
            uint32_t x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = (uint32_t)dense[(int64_t)(v + j) * K + k];
#pragma unroll
            for (int j = 0; j < 8; ++j) t += x[j];
        }
        for (; v < v1; ++v) t += (unsigned long long)(uint32_t)dense[(int64_t)v * K + k];
        if (t) atomicAdd(&out[k], t);
    }
}

hipError_t launch_row_sums(const int32_t *dense, int32_t V, int32_t K, unsigned long long *out, hipStream_t s)
{
    hipError_t e = launch_fill_u64(out, 0ull, K, s);
    if (e != hipSuccess) return e;
    row_sums_kernel<<<(V + ROWSUM_COLS - 1) / ROWSUM_COLS, 256, 0, s>>>(dense, V, K, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phi-step, part 1 (Section 3.4): one wave per word column v.
//   counted cells (n_kv = l >= 1) draw Pois(beta + l): alias table of l for
//   l <= L, rounded Gaussian for l > L;
//   zero-count cells draw Pois(beta); the nonzero ones are reached by
//   geometric jumps (gap = floor(-ln(1-U)/beta)), 64 jumps per round, their
//   positions by a wave prefix sum of the jump lengths.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) phi_draw_kernel(DevModel m, int32_t kpad)
{
    const uint32_t t = *m.tptr;
    extern __shared__ int32_t phi_lds[];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    const int32_t v = blockIdx.x * 4 + w;
    if (v >= m.V) return;
    int32_t *g = phi_lds + w * kpad;
    const int32_t K = m.K;
    const int32_t *ncol = m.n + (int64_t)v * K;
    const double two_pi = 6.283185307179586476925286766559;
    // per-word priors: the tables are of integer rates l and every cell's
    // Pois(beta_v) part comes from the prior marks below, added to its draw
    const bool vec = m.beta_v != nullptr;
    const double bv = vec ? m.beta_v[v] : m.beta;
    const double tb = vec ? 0.0 : m.beta;
    const uint32_t *T = m.ztp_tab + (vec ? m.ztp_off[v] : 0);
    const int32_t nT = vec ? m.ztp_off[v + 1] - m.ztp_off[v] : m.ztp_n;

    // counted cells, PR rounds of 64 cells at a time: the rounds' counts,
    // then their tables' offsets, then their alias entries are each loaded
    // for all rounds before any is used, so a column waits for three
    // dependent loads per PR rounds instead of per round
    constexpr int PR = 4;
    for (int32_t kb = 0; kb < K; kb += 64 * PR) {
        int32_t lv[PR];
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int32_t k = kb + 64 * u + lane;
            lv[u] = k < K ? ncol[k] : 0;
        }
        int32_t lo[PR], hi[PR];
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const bool tab = lv[u] > 0 && lv[u] <= m.L;
            lo[u] = tab ? m.pois_off[lv[u]] : 0;
            hi[u] = tab ? m.pois_off[lv[u] + 1] : 0;
        }
        int32_t x[PR];
        uint32_t jv[PR], ry[PR];
        uint64_t ev[PR];
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int32_t k = kb + 64 * u + lane;
            const int32_t l = lv[u];
            x[u] = -1;  // -1 marks a zero-count cell
            jv[u] = 0;
            ry[u] = 0;
            ev[u] = 0;
            if (l > 0) {
                const r4 r = philox((uint32_t)v, (uint32_t)k, t, TAG_PHI_CELL, m.key0, m.key1);
                if (l <= m.L) {
                    // alias table of rate l: slot j, kept when r.y is below
                    // its threshold, else its alias
                    jv[u] = scale32(r.x, (uint32_t)(hi[u] - lo[u]));
                    ry[u] = r.y;
                    ev[u] = m.pois[lo[u] + jv[u]];
                } else {
                    // rounded Gaussian of mean and variance lambda
                    const double lam = tb + (double)l;
                    const double rad = sqrt(-2.0 * log(1.0 - unit53(r.x, r.y)));
                    const double gz = rad * cos(two_pi * unit53(r.z, r.w));
                    const double y = floor(lam + sqrt(lam) * gz + 0.5);
                    x[u] = y > 0.0 ? (int32_t)y : 0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PR; ++u) {
            const int32_t k = kb + 64 * u + lane;
            const int32_t l = lv[u];
            if (l > 0 && l <= m.L) x[u] = (ry[u] < (uint32_t)ev[u]) ? (int32_t)jv[u] : (int32_t)(ev[u] >> 32);
            if (k < K) g[k] = x[u];
        }
    }
    __builtin_amdgcn_wave_barrier();

    long long pos_base = -1;
    for (uint32_t jb = 0;; jb += 64) {
        r4 r = philox((uint32_t)v, jb + (uint32_t)lane, t, TAG_PHI_PRIOR, m.key0, m.key1);
        const double e = -log(1.0 - unit53(r.x, r.y)) / bv;
        // a jump longer than K ends the column whatever its exact length
        const double capped = e < (double)K ? floor(e) : (double)K;
        const int32_t step = 1 + (int32_t)capped;
        const int32_t incl = group_scan_incl_i32<64>(step);
        const long long pos = pos_base + incl;
        if (pos < K) {
            int32_t *cell = &g[pos];
            int32_t x = 1;
            for (int q = 0; q < nT; ++q) x += (r.z >= T[q]) ? 1 : 0;
            if (*cell == -1) *cell = x;
            else if (vec) *cell += x;
        }
        const long long last = pos_base + __builtin_amdgcn_readlane(incl, 63);
        if (last >= K) break;
        pos_base = last;
    }
    __builtin_amdgcn_wave_barrier();

    int32_t cnt = 0;
    int32_t *gcol = m.gam + (int64_t)v * K;
    for (int32_t k = lane; k < K; k += 64) {
        int32_t x = g[k];
        x = x > 0 ? x : 0;
        gcol[k] = x;
        cnt += x > 0;
    }
    cnt = group_scan_incl_i32<64>(cnt);
    if (lane == 63) m.colcnt[v] = cnt;
}

// ---------------------------------------------------------------------------
// Phi-step, part 3: normalise (phi = fp32(gamma / S_k), quotient in fp64),
// write the dense tables and compact each column into the CSC (one wave per
// column, no LDS, so many columns are in flight); then build each column's
// alias table for the a-part (weights alpha_k phi_kv; Vose's construction
// with FIFO work lists in ascending order; sigma_a = ascending fp64 sum of
// the weights) from its compacted entries.
// DIR: Algorithm 1's Phi (fp64 Gamma draws gamd, fp64 row sums Sd): a cell
// is nonzero when its fp32 phi is normal (>= 2^-126), and every nonzero
// cell's 16-bit draw is the escape 0xFFFF (its phi is read from phid).
// ---------------------------------------------------------------------------
constexpr float FP32_MIN_NORMAL = 0x1p-126f;

template <bool DIR>
__global__ void __launch_bounds__(256) phi_dense_kernel(DevModel m)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= m.V) return;
    const int lane = __lane_id();
    const int32_t K = m.K;
    const int32_t cb = m.colptr[v];
    const int32_t *gcol = m.gam + (int64_t)v * K;
    const double *gdcol = m.gamd + (int64_t)v * K;
    float *pcol = m.phid + (int64_t)v * K;
    uint16_t *g16col = m.g16 + (int64_t)v * m.ks16;
    int32_t run = 0;
    float fmax = 0.0f;
    // the column's draws are read PB rounds of 64 cells at a time, so that
    // many loads are in flight before the rounds are processed in order
    constexpr int PB = 8;
    for (int32_t kb = 0; kb < m.ks16; kb += 64 * PB) {
    int32_t xs[PB];
    double gs[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) {
        const int32_t k = kb + 64 * j + lane;
        if constexpr (DIR) gs[j] = k < K ? gdcol[k] : 0.0;
        else xs[j] = k < K ? gcol[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < PB; ++j) {
        const int32_t k0 = kb + 64 * j;
        if (k0 >= m.ks16) break;
        const int32_t k = k0 + lane;
        float f = 0.0f;
        uint32_t x16 = 0;
        bool nz;
        if constexpr (DIR) {
            if (k < K && m.Sd[k] > 0.0) {
                f = (float)(gs[j] / m.Sd[k]);
                f = f >= FP32_MIN_NORMAL ? f : 0.0f;
            }
            nz = f > 0.0f;
            x16 = nz ? 0xFFFFu : 0u;
        } else {
            const int32_t x = xs[j];
            nz = x > 0;
            if (nz) f = (float)((double)x / (double)m.S[k]);
            const bool exact = x < 0xFFFF && (k >= K || m.S[k] < (1ull << 27));
            x16 = exact ? (uint32_t)x : 0xFFFFu;
        }
        if (k < K) pcol[k] = f;
        fmax = f > fmax ? f : fmax;
        g16col[k] = (uint16_t)x16;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(nz);
        if (nz) {
            const int32_t e = run + __builtin_popcountll(bal & ((1ull << lane) - 1ull));
            m.ctopic[cb + e] = (uint16_t)k;
            m.cphi[cb + e] = f;
            m.ckg[cb + e] = (uint32_t)k | (x16 << 16);
        }
        run += __builtin_popcountll(bal);
    }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const float y = __shfl_xor(fmax, o, 64);
        fmax = y > fmax ? y : fmax;
    }
    if (lane == 0) m.phimax[v] = fmax;
}

// Columns with at most ALIAS_SMALL nonzeros: one wave per column, four per
// block (LDS of ALIAS_SMALL entries each); the others: one column per block
// with K entries of LDS.  Per entry: a probability (fp64), a work-list
// entry (u16) and a turn mark (u8), so that many columns' chains run on a
// CU at once.
constexpr int32_t ALIAS_SMALL = 256;
constexpr size_t ALIAS_ENTRY_BYTES = sizeof(double) + sizeof(uint16_t) + sizeof(uint8_t);

template <bool SMALL>
__global__ void __launch_bounds__(SMALL ? 256 : 64) phi_alias_kernel(DevModel m, int32_t kpad)
{
    extern __shared__ double alias_lds[];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int32_t v = SMALL ? blockIdx.x * 4 + wave : blockIdx.x;
    if (v >= m.V) return;
    const int32_t cb = m.colptr[v];
    const int32_t nv = m.colptr[v + 1] - cb;
    if (SMALL ? nv > ALIAS_SMALL : nv <= ALIAS_SMALL) return;
    if (nv == 0) {
        if (lane == 0) m.sigma_a[v] = 0.0;
        return;
    }
    const int32_t cap = SMALL ? ALIAS_SMALL : kpad;
    // this wave's region: cap entries (cap is a multiple of 64, so every
    // region and array stays 8-byte aligned)
    double *pq = (double *)((uint8_t *)alias_lds + (size_t)wave * cap * ALIAS_ENTRY_BYTES);
    uint16_t *lst = (uint16_t *)(pq + cap);   // small entries from the front, large ones from the back
    uint8_t *mark = (uint8_t *)(lst + cap);   // 1 at the FIFO steps where the head turned small
    const uint16_t *ctop = m.ctopic + cb;     // topic of entry e
    // weights w_e = alpha_k phi_kv in entry order (pq holds them first;
    // each lane also keeps its first MAXC chunks' weights in registers, all
    // chunks' loads issued together)
    constexpr int MAXC = SMALL ? ALIAS_SMALL / 64 : 16;
    double wr[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int32_t e = c * 64 + lane;
        wr[c] = 0.0;
        if (e < nv) {
            wr[c] = m.alpha[ctop[e]] * (double)m.cphi[cb + e];
            pq[e] = wr[c];
        }
    }
    for (int32_t e = MAXC * 64 + lane; e < nv; e += 64) pq[e] = m.alpha[ctop[e]] * (double)m.cphi[cb + e];
    for (int32_t e = lane; e < nv; e += 64) mark[e] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // sigma_a: the ascending sum, read eight entries at a time
    double s = 0.0;
    if (lane == 0) {
        int32_t e = 0;
        for (; e + 8 <= nv; e += 8) {
            double b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) b[u] = pq[e + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += b[u];
        }
        for (; e < nv; ++e) s += pq[e];
        m.sigma_a[v] = s;
    }
    const double W = __shfl(s, 0, 64);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // p_e = w_e nv / W (w_e from registers: pq is reused); small
    // entries (p < 1) go to the front of lst in ascending order, large ones
    // to the back, the first large entry last; pq follows lst
    int32_t ns = 0, nl = 0;
    auto classify = [&](int32_t e, double w) {
        double p = 0.0;
        bool is_small = false;
        if (e < nv) {
            p = (w * (double)nv) / W;
            is_small = p < 1.0;
        }
        const uint64_t bs = __builtin_amdgcn_ballot_w64(e < nv && is_small);
        const uint64_t bl = __builtin_amdgcn_ballot_w64(e < nv && !is_small);
        const uint64_t below = (1ull << lane) - 1ull;
        if (e < nv) {
            const int32_t at = is_small ? ns + __builtin_popcountll(bs & below)
                                        : nv - 1 - (nl + __builtin_popcountll(bl & below));
            lst[at] = (uint16_t)e;
            pq[at] = p;
        }
        ns += __builtin_popcountll(bs);
        nl += __builtin_popcountll(bl);
    };
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
        if (c * 64 < nv) classify(c * 64 + lane, wr[c]);
    // chunks past MAXC (K > 64 MAXC) recompute their weights
    for (int32_t e0 = MAXC * 64; e0 < nv; e0 += 64) {
        const int32_t e = e0 + lane;
        classify(e, e < nv ? m.alpha[ctop[e]] * (double)m.cphi[cb + e] : 0.0);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // Vose's pairing.  The FIFO of small entries is the initial small list
    // followed by large entries in the order they turn small, and a large
    // entry can only turn small at the head of the large list, so both lists
    // are walked with one index each.  FIFO step f pairs small entry sm(f),
    // of probability ps(f), with the head of the large list: its threshold is
    // floor(ps(f) 2^32), its alias the large entry at the head, and the
    // head's probability becomes (pg + ps(f)) - 1; below 1 the head turns
    // small (its residual joins the FIFO) and the next large entry leads.
    // Only that chain of sums is sequential: lane 0 runs it and marks the
    // steps at which the head turned small (its residual goes to its own pq
    // slot); then all lanes write the records, the head at step f being
    // large entry number sum_{f' < f} mark[f'] (a prefix sum over the wave).
    int32_t nf = 0;
    if (lane == 0) {
        int32_t gi = 0, f = 0;
        double pg = nl > 0 ? pq[nv - 1] : 0.0;
        auto step = [&](double ps) {
            pg = (pg + ps) - 1.0;
            if (pg < 1.0) {
                pq[nv - 1 - gi] = pg;
                mark[f] = 1;
                ++gi;
                if (gi < nl) pg = pq[nv - 1 - gi];
            }
            ++f;
        };
        // the initial small entries, read eight at a time
        for (int32_t i = 0; i < ns && gi < nl; i += 8) {
            double pb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) pb[u] = pq[i + u < ns ? i + u : ns - 1];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i + u < ns && gi < nl) step(pb[u]);
        }
        // then the large entries that turned small, in that order
        while (gi < nl && f - ns < gi) step(pq[nv - 1 - (f - ns)]);
        nf = f;
    }
    nf = __shfl(nf, 0, 64);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // each entry's record: thr | topic << 32 | alias topic << 48.  The FIFO's
    // first nf entries are paired (threshold floor(ps 2^32), alias the head
    // at their step); the others keep themselves (threshold 2^32 - 1)
    uint64_t *rec = m.calias + cb;
    int32_t heads = 0;   // turns before this chunk of steps
    for (int32_t f0 = 0; f0 < nf; f0 += 64) {
        const int32_t f = f0 + lane;
        const int32_t mk = f < nf ? mark[f] : 0;
        const int32_t incl = group_scan_incl_i32<64>(mk);
        if (f < nf) {
            const int32_t at = f < ns ? f : nv - 1 - (f - ns);
            const int32_t sm = lst[at];
            const double ps = pq[at];
            const int32_t head = heads + incl - mk;
            const uint32_t al = lst[nv - 1 - head];
            rec[sm] = (uint64_t)(uint32_t)floor(ps * 4294967296.0) | ((uint64_t)ctop[sm] << 32) |
                      ((uint64_t)ctop[al] << 48);
        }
        heads += __builtin_amdgcn_readlane(incl, 63);
    }
    for (int32_t i = (nf < ns ? nf : ns) + lane; i < ns; i += 64) {
        const uint64_t k = ctop[lst[i]];
        rec[lst[i]] = 0xFFFFFFFFull | (k << 32) | (k << 48);
    }
    for (int32_t j = (nf > ns ? nf - ns : 0) + lane; j < nl; j += 64) {
        const int32_t sm = lst[nv - 1 - j];
        const uint64_t k = ctop[sm];
        rec[sm] = 0xFFFFFFFFull | (k << 32) | (k << 48);
    }
}

__global__ void word_records_kernel(DevModel m)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m.V) return;
    const int32_t cb = m.colptr[v];
    m.wrec[v] = make_uint4((uint32_t)cb, (uint32_t)(m.colptr[v + 1] - cb), __float_as_uint((float)m.sigma_a[v]),
                           __float_as_uint(m.phimax[v]));
}

hipError_t launch_word_records(const DevModel &m, hipStream_t s)
{
    word_records_kernel<<<(m.V + 255) / 256, 256, 0, s>>>(m);
    return hipGetLastError();
}

hipError_t launch_phi_fill(const DevModel &m, bool dir, hipStream_t s)
{
    if (dir) phi_dense_kernel<true><<<(m.V + 3) / 4, 256, 0, s>>>(m);
    else phi_dense_kernel<false><<<(m.V + 3) / 4, 256, 0, s>>>(m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t kpad = (m.K + 63) / 64 * 64;
    phi_alias_kernel<true><<<(m.V + 3) / 4, 256, 4 * ALIAS_SMALL * ALIAS_ENTRY_BYTES, s>>>(m, kpad);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m.K > ALIAS_SMALL) {
        phi_alias_kernel<false><<<m.V, 64, (size_t)kpad * ALIAS_ENTRY_BYTES, s>>>(m, kpad);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_word_records(m, s);
}

__global__ void colptr_finish_kernel(const unsigned long long *S, int32_t K, const long long *total,
                                     unsigned long long *stats, double *Rd)
{
    if (threadIdx.x == 0 && stats) {
        stats[ST_NNZ_PHI] = (unsigned long long)*total;
    }
    unsigned long long empty = 0;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        empty += S[k] == 0;
        Rd[k] = S[k] ? 1.0 / (double)S[k] : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) empty += __shfl_down(empty, o, 64);
    if ((threadIdx.x & 63) == 0 && empty && stats) atomicAdd(&stats[ST_EMPTY_ROWS], empty);
}

hipError_t launch_phi_step(const DevModel &m, unsigned long long *stats, hipStream_t s)
{
    const int32_t kpad = (m.K + 63) / 64 * 64;
    phi_draw_kernel<<<(m.V + 3) / 4, 256, 4 * kpad * sizeof(int32_t), s>>>(m, kpad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_row_sums(m.gam, m.V, m.K, m.S, s);
    if (e != hipSuccess) return e;
    long long *scratch = m.scratch;
    long long *total = scratch + ((m.V + SCAN_BLOCK - 1) / SCAN_BLOCK) + 1;
    e = scan_excl<int32_t, int32_t>(m.colcnt, m.colptr, m.V, scratch, total, s);
    if (e != hipSuccess) return e;
    if (stats) {
        e = launch_fill_u64(&stats[ST_EMPTY_ROWS], 0ull, 1, s);
        if (e != hipSuccess) return e;
    }
    colptr_finish_kernel<<<1, 256, 0, s>>>(m.S, m.K, total, stats, m.Rd);
    return launch_phi_fill(m, false, s);
}

// ---------------------------------------------------------------------------
// Algorithm 1's Phi-step: phi_k ~ Dir(n_k + beta) for every topic row, by
// the Gamma representation of the Dirichlet (Section 3.3): gamma_kv ~
// G(beta + n_kv, 1) and phi_kv = gamma_kv / S_k with S_k = sum_v gamma_kv.
// Gamma draws by Marsaglia and Tsang's method, which Section 3.4 names: for
// shape a >= 1, d = a - 1/3 and c = 1 / sqrt(9 d), a normal x gives
// t = 1 + c x (rejected when t <= 0) and v = t^3, kept as d v when a
// uniform u passes their squeeze u < 1 - 0.0331 x^4 or
// log u < x^2 / 2 + d (1 - v + log v); shapes below 1 use their boost
// G(a) = G(a + 1) U^(1/a), U^(1/a) taken as exp(log(U) / a).
// Attempt j of cell (k, v) at sweep t reads Philox counter
// (v, k, t, TAG_PHI_GAMMA + 256 j): the normal is Box-Muller's
// sqrt(-2 log u(r0)) cos(2 pi u(r1)), u = u(r2), and r3 of attempt 0 is the
// boost's U, with u(r) = (r + 1/2) 2^-32.  After 2^20 rejected attempts
// (probability below 0.05^(2^20)) the draw is d.
// ---------------------------------------------------------------------------
constexpr uint32_t GAMMA_TRIES = 1u << 20;

__device__ __forceinline__ double unit32o(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

__device__ double gamma_draw(double a, uint32_t c0, uint32_t c1, uint32_t t, uint32_t key0, uint32_t key1)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double a1 = a < 1.0 ? a + 1.0 : a;
    const double d = a1 - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double g = d;
    uint32_t boost = 0;
    for (uint32_t j = 0; j < GAMMA_TRIES; ++j) {
        const r4 r = philox(c0, c1, t, TAG_PHI_GAMMA + (j << 8), key0, key1);
        if (j == 0) boost = r.w;
        const double x = sqrt(-2.0 * log(unit32o(r.x))) * cos(two_pi * unit32o(r.y));
        const double t1 = 1.0 + c * x;
        if (t1 <= 0.0) continue;
        const double v = t1 * t1 * t1;
        const double u = unit32o(r.z);
        const double x2 = x * x;
        if (u < 1.0 - 0.0331 * (x2 * x2) || log(u) < 0.5 * x2 + d * (1.0 - v + log(v))) {
            g = d * v;
            break;
        }
    }
    if (a < 1.0) g = g * exp(log(unit32o(boost)) / a);
    return g;
}

// one cell per thread, word-major (cell v * K + k)
__global__ void __launch_bounds__(256) gamma_kernel(DevModel m)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cells = (int64_t)m.V * m.K;
    if (cell >= cells) return;
    const uint32_t t = *m.tptr;
    const int32_t v = (int32_t)(cell / m.K);
    const int32_t k = (int32_t)(cell - (int64_t)v * m.K);
    const double a = (m.beta_v ? m.beta_v[v] : m.beta) + (double)m.n[cell];
    m.gamd[cell] = gamma_draw(a, (uint32_t)v, (uint32_t)k, t, m.key0, m.key1);
}

// S_k in two fixed-order passes (so the Phi-step is deterministic): block b
// sums its ROWSUM_COLS words in ascending order per topic, then the blocks'
// partial sums are added in ascending block order
__global__ void dsum_part_kernel(DevModel m)
{
    const int32_t v0 = blockIdx.x * ROWSUM_COLS;
    const int32_t v1 = v0 + ROWSUM_COLS < m.V ? v0 + ROWSUM_COLS : m.V;
    for (int32_t k = threadIdx.x; k < m.K; k += blockDim.x) {
        double s = 0.0;
        for (int32_t v = v0; v < v1; ++v) s += m.gamd[(int64_t)v * m.K + k];
        m.dpart[(int64_t)blockIdx.x * m.K + k] = s;
    }
}

__global__ void dsum_final_kernel(DevModel m, int32_t nb)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m.K) return;
    double s = 0.0;
    for (int32_t b = 0; b < nb; ++b) s += m.dpart[(int64_t)b * m.K + k];
    m.Sd[k] = s;
}

// nonzeros of each column: cells whose fp32 phi is normal; one wave per word
__global__ void __launch_bounds__(256) dcount_kernel(DevModel m)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= m.V) return;
    const int lane = __lane_id();
    const double *gdcol = m.gamd + (int64_t)v * m.K;
    int32_t cnt = 0;
    for (int32_t k = lane; k < m.K; k += 64) {
        const double S = m.Sd[k];
        const float f = S > 0.0 ? (float)(gdcol[k] / S) : 0.0f;
        cnt += f >= FP32_MIN_NORMAL;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) m.colcnt[v] = cnt;
}

__global__ void dcolptr_finish_kernel(const double *Sd, int32_t K, const long long *total,
                                      unsigned long long *stats, double *Rd)
{
    if (threadIdx.x == 0 && stats) stats[ST_NNZ_PHI] = (unsigned long long)*total;
    unsigned long long empty = 0;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) {
        empty += Sd[k] == 0.0;
        Rd[k] = 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) empty += __shfl_down(empty, o, 64);
    if ((threadIdx.x & 63) == 0 && empty && stats) atomicAdd(&stats[ST_EMPTY_ROWS], empty);
}

hipError_t launch_phi_step_dirichlet(const DevModel &m, unsigned long long *stats, hipStream_t s)
{
    if (m.phi_method != 1) return hipErrorInvalidValue;
    const int64_t cells = (int64_t)m.V * m.K;
    gamma_kernel<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t nb = (m.V + ROWSUM_COLS - 1) / ROWSUM_COLS;
    dsum_part_kernel<<<nb, 256, 0, s>>>(m);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dsum_final_kernel<<<(m.K + 255) / 256, 256, 0, s>>>(m, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dcount_kernel<<<(m.V + 3) / 4, 256, 0, s>>>(m);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    long long *scratch = m.scratch;
    long long *total = scratch + ((m.V + SCAN_BLOCK - 1) / SCAN_BLOCK) + 1;
    e = scan_excl<int32_t, int32_t>(m.colcnt, m.colptr, m.V, scratch, total, s);
    if (e != hipSuccess) return e;
    if (stats) {
        e = launch_fill_u64(&stats[ST_EMPTY_ROWS], 0ull, 1, s);
        if (e != hipSuccess) return e;
    }
    dcolptr_finish_kernel<<<1, 256, 0, s>>>(m.Sd, m.K, total, stats, m.Rd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_phi_fill(m, true, s);
}

// ---------------------------------------------------------------------------
// z-step (Section 3.5).  A group of G lanes (G = 8, 16, 32, 64) owns one
// document at a time and walks its tokens in stored order (sequential Gibbs
// within the document).  The document-topic counts m_d live in LDS, indexed
// by topic, beside lst, the document's topics with a nonzero count in
// ascending order.  For each token:
//   sigma_b = sum_k phi_kv m_k is taken over the document's topics (lst,
//   phi from the word's dense column of draws) or the word's Phi column
//   (its CSC entries, m from LDS); either way lane g takes a contiguous
//   block of entries in ascending topic order and a group prefix sum orders
//   the lanes, so the running sums are ascending in k as the definition
//   requires;
//   u_sigma = u (sigma_a + sigma_b) < sigma_a takes the word's alias draw,
//   otherwise the crossing lane (first with prefix > u_sigma - sigma_a)
//   walks its entries to find the topic;
//   the counts and lst are updated: a topic that leaves or enters the
//   document moves the entries above it by one place.
// ---------------------------------------------------------------------------
struct ZArgs {
    DevModel m;
    DevCorpus c;
    const WorkItem *items;
    int32_t n_items;
    int32_t m_bytes;           // count table of one group
    int32_t group_bytes;       // count table and topic list of one group
    int32_t wave_bytes;        // the groups of one wave
    int32_t r_bytes;           // the block's copy of R_k, at the start of LDS
    int32_t n_hot;             // frequent words counted per block in LDS (0: none)
    int32_t hot_off;           // their counters' byte offset in LDS
    int32_t *queue;
    unsigned long long *stats;
    double *ll_doc;         // per-document log-joint terms (or null)
};

// inputs of one token draw, staged in LDS so every lane of the group reads
// them with one broadcast load
struct alignas(16) TokenIn {
    uint32_t vk;     // v * K: the word's row of n and of the dense phi
    int32_t cb;      // first CSC entry of the word's Phi column
    uint16_t kold;   // topic before the draw
    uint16_t kv;     // nonzeros in the column (K_v^Phi <= K <= 4096)
    float u0;        // the 24-bit uniform of the a/b decision and the b-walk
                     // (r >> 8) 2^-24, exact in fp32
    uint16_t ka;     // the a-part's topic: the alias draw depends only on the
                     // word and the token's random numbers, so it is taken at
                     // staging time, off the draw's critical path
    uint16_t sure;   // 1: the a-part is certain whatever the document's counts
    uint32_t vs;     // v * ks16: the word's row of the 16-bit draws (the
                     // products are taken once, at staging)
    double sa;       // sigma_a(v)
};

static_assert(sizeof(TokenIn) == 32, "TokenIn is staged as 32-byte records");

// the z-step's staged token: as TokenIn, with sigma_a in fp32 (its fp32
// b-part) and the word id (the fp64 b-part reads sigma_a(v) itself)
struct alignas(16) TokenZ {
    uint32_t vk;     // v * K
    int32_t cb;      // first CSC entry of the word's Phi column
    uint16_t kold;   // topic before the draw
    uint16_t kv;     // nonzeros in the column
    float u0;        // (r0 >> 8) 2^-24
    uint16_t ka;     // the a-part's alias draw
    uint16_t sure;   // 1: the a-part is certain whatever the document's counts
    uint32_t vs;     // v * ks16
    float saf;       // fp32(sigma_a(v))
    uint32_t v;      // the word
};

static_assert(sizeof(TokenZ) == 32, "TokenZ is staged as 32-byte records");

// draw statistics of a lane's group: totals, and the current document's J
// and a-part counts in 32 bits (cheaper to add per draw), moved into the
// totals when the document is done
struct ZCount {
    unsigned long long J, A, degenerate;
    uint32_t j, a;
    __device__ void flush()
    {
        J += j;
        A += a;
        j = 0;
        a = 0;
    }
};

// the z-step's draw statistics of the current document (group-uniform,
// 32-bit), added to the wave's 64-bit totals in LDS when the document is
// done: sum of J, the same over the tokens whose b-terms were computed (not
// decided at staging), a-part draws, degenerate tokens
struct ZCount32 {
    uint32_t j, jb, a, deg, fb;   // fb: draws the fp32 b-part left to the fp64 one
};

// b-terms per lane kept in registers for the walk: one gather round covers
// G * keep entries
template <int G>
constexpr int keep_of()
{
    return G <= 8 ? 8 : 4;
}

template <int G>
constexpr int log2g()
{
    return G == 64 ? 6 : (G == 32 ? 5 : (G == 16 ? 4 : 3));
}

// list slots per lane in the windowed topic list: W G slots hold the list
// while it is no longer than that (128 for groups of 16 and 32)
template <int G>
constexpr int win_of()
{
    return G == 16 ? 8 : 4;
}

// value of the windowed list's slots past its end: above every topic
// (K <= 4096) and below 2^15, so that packed signed 16-bit differences of
// slot values never overflow
constexpr int32_t LIST_PAD = 0x7FFF;

// The state of the document a group is working on: m_d by topic (mt) and
// lst, its topics with a nonzero count in ascending order (during a draw it
// also holds the token's old topic, whose count may be zero: that b-term is
// zero).  lst[0] always holds a valid topic, so padding slots can read it.
// WIN: lst is 16-byte aligned and has room for W G + W slots (W =
// win_of<G>()), and every slot in [L, W G + W) holds LIST_PAD (see
// list_window_update).
template <typename CT, bool WIN = false>
struct DocState {
    CT *mt;
    uint16_t *lst;
    int32_t L;       // entries of lst (group-uniform)
};

// lst <- the topics with a nonzero count; lane g scans topics [g*R, g*R + R)
template <int G, typename CT, bool WIN>
__device__ __forceinline__ void build_list(DocState<CT, WIN> &S, int g, int32_t K)
{
    if constexpr (WIN) {
        // the windows read LIST_PAD past the list
        constexpr int W = win_of<G>();
        const uint32_t pad2 = (uint32_t)LIST_PAD * 0x10001u;
#pragma unroll
        for (int j = 0; j < W; j += 2) *(uint32_t *)(S.lst + W * g + j) = pad2;
        if (g == 0) {
#pragma unroll
            for (int j = 0; j < W; j += 2) *(uint32_t *)(S.lst + W * G + j) = pad2;
        }
        __builtin_amdgcn_wave_barrier();
    }
    const int32_t R = (K + G - 1) / G;
    const int32_t t0 = g * R;
    const int32_t t1 = t0 + R < K ? t0 + R : K;
    int32_t c = 0;
    for (int32_t t = t0; t < t1; ++t) c += S.mt[t] != 0;
    const int32_t incl = group_scan_incl_i32<G>(c);
    int32_t o = incl - c;
    S.L = group_bcast<G>(incl, G - 1);
    for (int32_t t = t0; t < t1; ++t)
        if (S.mt[t]) S.lst[o++] = (uint16_t)t;
    __builtin_amdgcn_wave_barrier();
}

// lane g's block of lst: entries [base, base + n), q = ceil(L / G) per lane
template <int G>
__device__ __forceinline__ int32_t list_block(int32_t L, int g, int32_t &base)
{
    const int32_t q = (L + G - 1) / G;
    base = (int32_t)__umul24((uint32_t)g, (uint32_t)q);
    const int32_t n = L - base < q ? L - base : q;
    return n > 0 ? n : 0;
}

// insert topic k (not in lst): the entries above it move up one place
template <int G, typename CT, bool WIN>
__device__ __forceinline__ void list_insert(DocState<CT, WIN> &S, int32_t k, int g)
{
    int32_t base;
    const int32_t n = list_block<G>(S.L, g, base);
    // the block's first entry is overwritten by the lane below: read it first
    const int32_t first = n > 0 ? S.lst[base] : 0;
    __builtin_amdgcn_wave_barrier();
    int32_t below = 0;
    for (int32_t j = n - 1; j >= 1; --j) {
        const int32_t v = S.lst[base + j];
        if (v > k) S.lst[base + j + 1] = (uint16_t)v;
        else ++below;
    }
    if (n > 0) {
        if (first > k) S.lst[base + 1] = (uint16_t)first;
        else ++below;
    }
    const int32_t pos = group_bcast<G>(group_scan_incl_i32<G>(below), G - 1);
    __builtin_amdgcn_wave_barrier();
    if (g == 0) S.lst[pos] = (uint16_t)k;
    S.L += 1;
    __builtin_amdgcn_wave_barrier();
}

// remove topic k (in lst): the entries above it move down one place
template <int G, typename CT, bool WIN>
__device__ __forceinline__ void list_remove(DocState<CT, WIN> &S, int32_t k, int g)
{
    int32_t base;
    const int32_t n = list_block<G>(S.L, g, base);
    // the block's last entry is overwritten by the lane above: read it first
    const int32_t last = n > 0 ? S.lst[base + n - 1] : 0;
    __builtin_amdgcn_wave_barrier();
    for (int32_t j = 0; j < n; ++j) {
        const int32_t v = j == n - 1 ? last : S.lst[base + j];
        if (v > k) S.lst[base + j - 1] = (uint16_t)v;
    }
    S.L -= 1;
    // the slot freed at the end reads LIST_PAD again
    if constexpr (WIN)
        if (g == 0) S.lst[S.L] = (uint16_t)LIST_PAD;
    __builtin_amdgcn_wave_barrier();
}

// The list as windows of W slots: lane g of the group holds slots
// [W g, W g + W), W/2 32-bit LDS words of two slots each.  While every entry
// lies inside the windows (L <= W G before and after), removing kout and
// inserting kin (LIST_PAD: nothing) take one pass: each lane reads its window
// and the slot on either side, forms its new window in registers and writes
// it back.  Slots past the list hold LIST_PAD, so the same rules cover the
// list's end.  With o the old slots (ascending) the two steps are
//   removal:   o'[j] = o[j] < kout ? o[j] : o[j+1]
//              = min(max(o[j], M_j), o[j+1]),  M_j = (o[j] >= kout) ? 0xFFFF : 0
//   insertion: o''[j] = min(o'[j], max(o'[j-1], kin))
// (for a sorted list the first entry not below kin takes kin and the ones
// above it take their left neighbour), evaluated two slots at a time with
// packed 16-bit min, max, subtract and shift.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

template <int W>
struct alignas(2 * W) WinWords {
    uint32_t w[W / 2];
};

template <int G, typename CT, bool WIN>
__device__ __forceinline__ void list_window_update(DocState<CT, WIN> &S, int32_t kout, int32_t kin, int g)
{
    static_assert(WIN, "the windows need the padded list");
    constexpr int W = win_of<G>();
    constexpr int NW = W / 2;
    uint16_t *w = S.lst + W * g;
    WinWords<W> cur = *(const WinWords<W> *)w;
    // (lane 0 reads the slot before the list, inside the count table, and
    // drops it: an unconditional read needs no lane mask)
    const uint32_t lraw = w[-1];
    const uint32_t left = g > 0 ? lraw : 0u;
    const uint32_t right = w[W];
    __builtin_amdgcn_wave_barrier();
    // removal (kout - 1 wraps to 0xFFFF for kout = 0: every slot moves)
    const u16x2 km1 = (u16x2)(unsigned short)(kout - 1);
    uint32_t r[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t nxt = __builtin_amdgcn_alignbit(i + 1 < NW ? cur.w[i + 1] : right, cur.w[i], 16);
        const u16x2 a = as_u16x2(cur.w[i]);
        const u16x2 m = __builtin_bit_cast(u16x2, __builtin_bit_cast(i16x2, km1 - a) >> (i16x2)15);
        r[i] = as_u32(__builtin_elementwise_min(__builtin_elementwise_max(a, m), as_u16x2(nxt)));
    }
    // the new value of the slot left of the window
    const uint32_t o0 = cur.w[0] & 0xFFFFu;
    const uint32_t p = (int32_t)left < kout ? left : o0;
    // insertion
    const u16x2 kin2 = (u16x2)(unsigned short)kin;
    WinWords<W> out;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t prv = __builtin_amdgcn_alignbit(r[i], i > 0 ? r[i - 1] : p << 16, 16);
        out.w[i] = as_u32(__builtin_elementwise_min(as_u16x2(r[i]), __builtin_elementwise_max(as_u16x2(prv), kin2)));
    }
    *(WinWords<W> *)w = out;
    __builtin_amdgcn_wave_barrier();
}

// after a draw: the old topic leaves the list when its count fell to zero,
// the new one enters when it was absent
template <int G, typename CT, bool WIN>
__device__ __forceinline__ void list_update(DocState<CT, WIN> &S, int32_t kold, int32_t knew, int32_t mo,
                                            int32_t mn, int g)
{
    const bool out = knew != kold && mo == 1;
    const bool in = knew != kold && mn == 0;
    if constexpr (WIN) {
        if (__builtin_amdgcn_ballot_w64(out || in) == 0) return;
        constexpr int32_t CAP = win_of<G>() * G;
        const int32_t L2 = S.L + (in ? 1 : 0) - (out ? 1 : 0);
        const bool wide = (out || in) && (S.L > CAP || L2 > CAP);
        if (__builtin_amdgcn_ballot_w64(wide) == 0) {
            list_window_update<G>(S, out ? kold : LIST_PAD, in ? knew : LIST_PAD, g);
            S.L = L2;
            return;
        }
    }
    if (out) list_remove<G>(S, kold, g);
    if (in) list_insert<G>(S, knew, g);
}

// up to KP b-terms of this lane: entries first + base + u (u < KP) of its
// block, which has nl entries: topic, phi and m_d of each (count zeroed
// past the end).  DOC: the block is in the document's topic list (LDS) and
// the draw is gathered from the word's dense 16-bit column; otherwise the
// block is of the word's packed CSC entries (topic | draw << 16), read
// contiguously.  R (LDS) holds R_k.  Every slot loads from a valid address
// (padding slots read entry `pad`), so all loads of a round are in flight
// together.
// Global reads take a 32-bit byte offset from the table's base (the plan
// keeps every table under 4 GiB), so each address is one 32-bit add.
template <typename T>
__device__ __forceinline__ T load_at(const T *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}

template <int KP, bool DOC, typename CT>
__device__ __forceinline__ void lane_terms(const DevModel &M, const uint16_t *lst, const uint32_t g16o,
                                           const uint32_t vk, const double *R, const CT *mt, const int32_t pad,
                                           const int32_t first, const int32_t base, const int32_t nl,
                                           int32_t (&kk)[KP], float (&fk)[KP], int32_t (&mk)[KP])
{
    bool ok[KP];
    uint32_t x[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        ok[u] = base + u < nl;
        const uint32_t e = (uint32_t)(ok[u] ? first + base + u : pad);
        if constexpr (DOC) {
            kk[u] = lst[e];
        } else {
            const uint32_t kg = load_at(M.ckg, e << 2);
            kk[u] = (int32_t)(kg & 0xFFFFu);
            x[u] = kg >> 16;
        }
    }
    if constexpr (DOC) {
        if (M.phi_method == 1) {
            // Algorithm 1's Phi has no integer draws: phi itself is gathered
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                fk[u] = load_at(M.phid, (vk + (uint32_t)kk[u]) << 2);
                const int32_t m = mt[kk[u]];
                mk[u] = ok[u] ? m : 0;
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) x[u] = load_at(M.g16, g16o + ((uint32_t)kk[u] << 1));
    }
    // phi_kv = fp32(x * R_k) == fp32(RN64(x / S_k)) for x < 2^16 and
    // S_k < 2^27; every other nonzero cell carries 0xFFFF and its phi is
    // read from the dense table (rare: one wave-uniform test per round)
    bool esc = false;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const double r = R[kk[u]];
        const int32_t m = mt[kk[u]];
        fk[u] = (float)((double)x[u] * r);
        esc |= x[u] == 0xFFFFu;
        mk[u] = ok[u] ? m : 0;
    }
    if (__builtin_amdgcn_ballot_w64(esc)) {
#pragma unroll
        for (int u = 0; u < KP; ++u)
            if (x[u] == 0xFFFFu) fk[u] = load_at(M.phid, (vk + (uint32_t)kk[u]) << 2);
    }
}

// sigma_b = sum of the b-terms phi_kv m_k over one side, the a/b decision,
// and for the b-part the topic whose running sum first exceeds
// y = u_sigma - sigma_a (Section 3.5).  Returns the topic, or -1 for the
// a-part (the caller takes the word's alias draw).  KP terms per lane and
// round; the first round's terms stay in registers for the walk.
template <int G, bool DOC, typename CT, int KP, bool WIN>
__device__ __forceinline__ int32_t b_part(const DevModel &M, const TokenIn &tk, DocState<CT, WIN> &S, const double *R,
                                          const int g, double &Zo)
{
    constexpr int LG = log2g<G>();
    const int32_t J = DOC ? S.L : (int32_t)tk.kv;
    const int32_t q = (J + G - 1) >> LG;
    int32_t nl = J - g * q < q ? J - g * q : q;
    nl = nl > 0 ? nl : 0;
    const uint32_t g16o = tk.vs << 1;
    const int32_t pad = DOC ? 0 : tk.cb;
    const int32_t first = pad + (int32_t)__umul24((uint32_t)g, (uint32_t)q);
    int32_t kk[KP], mk[KP];
    float fk[KP];
    lane_terms<KP, DOC, CT>(M, S.lst, g16o, tk.vk, R, S.mt, pad, first, 0, nl, kk, fk, mk);
    // the products phi * m are exact in fp64, so adding them (or an fma)
    // rounds exactly like the sum of the products
    double bk[KP];
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        bk[u] = (double)fk[u] * (double)mk[u];
        p += bk[u];
    }
    for (int32_t base = KP; base < nl; base += KP) {
        int32_t k2[KP], m2[KP];
        float f2[KP];
        lane_terms<KP, DOC, CT>(M, S.lst, g16o, tk.vk, R, S.mt, pad, first, base, nl, k2, f2, m2);
#pragma unroll
        for (int u = 0; u < KP; ++u) p = __builtin_fma((double)f2[u], (double)m2[u], p);
    }
    const double incl = group_scan_incl<G>(p);
    const double T = group_bcast_f64<G>(incl, G - 1);
    const double Z = tk.sa + T;
    Zo = Z;
    const double x = (double)tk.u0 * Z;
    if (x < tk.sa) return -1;
    // b-part: the first lane whose running sum passes y walks its terms
    const double y = x - tk.sa;
    const uint64_t bal = group_ballot<G>(incl > y);
    int f = -1;
    if (bal) {
        f = G <= 32 ? __builtin_ctz((uint32_t)bal) : __builtin_ctzll(bal);
    } else {
        const uint64_t pos = group_ballot<G>(p > 0.0);
        if (pos) f = 63 - __builtin_clzll(pos);
    }
    if (f < 0) return -1;  // no positive b-term survived rounding: the a-part is the whole law
    // every lane walks its kept terms (registers only, no branch around the
    // crossing lane); the crossing lane's result is the draw, unless its
    // block holds more terms than were kept: then that lane walks them all
    int32_t kf = -1;
    {
        double c = incl - p;
        int32_t last = -1;
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            if (bk[u] > 0.0) {
                c += bk[u];
                last = kk[u];
                if (kf < 0 && c > y) kf = kk[u];
            }
        }
        if (kf < 0) kf = last;
    }
    if (nl > KP && g == f) {
        double c = incl - p;
        int32_t last = -1;
        kf = -1;
        {
            for (int32_t base = 0; base < nl && kf < 0; base += KP) {
                int32_t k2[KP], m2[KP];
                float f2[KP];
                lane_terms<KP, DOC, CT>(M, S.lst, g16o, tk.vk, R, S.mt, pad, first, base, nl, k2, f2, m2);
#pragma unroll
                for (int u = 0; u < KP; ++u) {
                    const double bv = (double)f2[u] * (double)m2[u];
                    if (bv > 0.0) {
                        c += bv;
                        last = k2[u];
                        if (kf < 0 && c > y) kf = k2[u];
                    }
                }
            }
        }
        if (kf < 0) kf = last;
    }
    return group_bcast<G>(kf, f);
}

// ---------------------------------------------------------------------------
// The same b-part in fp32 with a proven error bound, the z-step's common
// path.  Every quantity is within a known relative error of its exact value:
// a term b~ = fp32(fp32(x R~_k) m) (R~_k = fp32(R_k)) or fp32(phi m) is
// within 4.01 u of phi_kv m_k (u = 2^-24), a lane's partial sum of q terms
// adds (q - 1) u, the group scan log2(G) u and the exclusive prefix u
// (relative to sigma_b), and the walk over the crossing lane's terms q u
// more.  x = u0 (sigma_a + sigma_b) and y = x - sigma_a are within
// (q + 8 + log2 G) u Z of their exact values, so every comparison of y with
// 0 or with a running sum errs by less than (3q + 2 log2 G + 13) u Z.  The
// decision is taken here only when y lies farther than
// tol = (64 + 8q) u Z from the boundary it is compared with (at least 2.4
// times that error); it is then the exact-arithmetic decision, which is also
// the fp64 path's (b_part).  Otherwise (returned as -2; the z-step counts
// these draws: about 5e-4 per token on a 1000-topic corpus) the caller runs
// b_part.  So the result is b_part's bit for bit.
// Returns the topic, -1 for the a-part or -2 for undecided.
// ---------------------------------------------------------------------------
template <int KP, bool DOC, typename CT, bool EARLY>
__device__ __forceinline__ void lane_terms_f32(const DevModel &M, const uint16_t *lst, const uint32_t g16o,
                                               const uint32_t vk, const float *Rf, const CT *mt, const int32_t pad,
                                               const int32_t first, const int32_t base, const int32_t nl,
                                               int32_t (&kk)[KP], float (&bf)[KP])
{
    bool ok[KP];
    uint32_t x[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        ok[u] = base + u < nl;
        const uint32_t e = (uint32_t)(ok[u] ? first + base + u : pad);
        if constexpr (DOC) {
            kk[u] = lst[e];
        } else {
            const uint32_t kg = load_at(M.ckg, e << 2);
            kk[u] = (int32_t)(kg & 0xFFFFu);
            x[u] = kg >> 16;
        }
    }
    if constexpr (DOC) {
        if (M.phi_method == 1) {
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                const float f = load_at(M.phid, (vk + (uint32_t)kk[u]) << 2);
                const int32_t m = mt[kk[u]];
                bf[u] = f * (float)(ok[u] ? m : 0);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < KP; ++u) x[u] = load_at(M.g16, g16o + ((uint32_t)kk[u] << 1));
    }
    // each term's R_k and count (LDS).  EARLY: all issued before any
    // gathered draw is used; left to itself the scheduler waits for the
    // first gather before the later terms' LDS reads, adding their latency
    // to the gathers' (the z-step's long documents draw 4% faster so; the
    // fold-in kernel, which passes false, 2% slower)
    float rr[KP];
    int32_t mm[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        rr[u] = Rf[kk[u]];
        mm[u] = mt[kk[u]];
    }
    if constexpr (EARLY) __builtin_amdgcn_sched_barrier(0);
    bool esc = false;
    float mf[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        mf[u] = (float)(ok[u] ? mm[u] : 0);
        bf[u] = ((float)x[u] * rr[u]) * mf[u];
        esc |= x[u] == 0xFFFFu;
    }
    if (__builtin_amdgcn_ballot_w64(esc)) {
#pragma unroll
        for (int u = 0; u < KP; ++u)
            if (x[u] == 0xFFFFu) bf[u] = load_at(M.phid, (vk + (uint32_t)kk[u]) << 2) * mf[u];
    }
}

template <int G, bool DOC, typename CT, int KP, bool WIN, bool EARLY>
__device__ __forceinline__ int32_t b_part_f32(const DevModel &M, const TokenZ &tk, DocState<CT, WIN> &S,
                                              const float *Rf, const int g)
{
    constexpr int LG = log2g<G>();
    const int32_t J = DOC ? S.L : (int32_t)tk.kv;
    const int32_t q = (J + G - 1) >> LG;
    int32_t nl = J - g * q < q ? J - g * q : q;
    nl = nl > 0 ? nl : 0;
    const uint32_t g16o = tk.vs << 1;
    const int32_t pad = DOC ? 0 : tk.cb;
    const int32_t first = pad + (int32_t)__umul24((uint32_t)g, (uint32_t)q);
    int32_t kk[KP];
    float bf[KP];
    lane_terms_f32<KP, DOC, CT, EARLY>(M, S.lst, g16o, tk.vk, Rf, S.mt, pad, first, 0, nl, kk, bf);
    float p = 0.0f;
#pragma unroll
    for (int u = 0; u < KP; ++u) p += bf[u];
    for (int32_t base = KP; base < nl; base += KP) {
        int32_t k2[KP];
        float f2[KP];
        lane_terms_f32<KP, DOC, CT, EARLY>(M, S.lst, g16o, tk.vk, Rf, S.mt, pad, first, base, nl, k2, f2);
#pragma unroll
        for (int u = 0; u < KP; ++u) p += f2[u];
    }
    const float incl = group_scan_incl_f32<G>(p);
    const float T = group_bcast_f32<G>(incl, G - 1);
    const float sa = tk.saf;
    const float Z = sa + T;
    const float y = tk.u0 * Z - sa;
    const float tol = Z * ((float)(64 + 8 * q) * 0x1p-24f);
    // (a sigma_a too small for fp32's normal range goes to the fp64 path)
    if (y < -tol && sa > 0x1p-100f) return -1;
    if (!(y > tol) || !(sa > 0x1p-100f)) return -2;
    const uint64_t bal = group_ballot<G>(incl > y);
    if (!bal) return -2;
    const int f = G <= 32 ? __builtin_ctz((uint32_t)bal) : __builtin_ctzll(bal);
    // every lane walks its kept terms; the crossing lane's result is the
    // draw when its interval [lo, hi) keeps tol from y on both sides
    float c = incl - p;
    int32_t kf = -1;
    float lo = 0.0f, hi = 0.0f;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
        const float c2 = c + bf[u];
        if (kf < 0 && bf[u] > 0.0f && c2 > y) {
            kf = kk[u];
            lo = c;
            hi = c2;
        }
        c = c2;
    }
    if (nl > KP && g == f && kf < 0) {
        for (int32_t base = KP; base < nl && kf < 0; base += KP) {
            int32_t k2[KP];
            float f2[KP];
            lane_terms_f32<KP, DOC, CT, EARLY>(M, S.lst, g16o, tk.vk, Rf, S.mt, pad, first, base, nl, k2, f2);
#pragma unroll
            for (int u = 0; u < KP; ++u) {
                const float c2 = c + f2[u];
                if (kf < 0 && f2[u] > 0.0f && c2 > y) {
                    kf = k2[u];
                    lo = c;
                    hi = c2;
                }
                c = c2;
            }
        }
    }
    const int32_t res = (kf >= 0 && y - lo > tol && hi - y > tol) ? kf : -2;
    return group_bcast<G>(res, f);
}

// draw one token (group-uniform control flow); returns the new topic, or
// -1 - kold for a token whose word has an empty Phi column (it keeps kold)
template <int G, typename CT, bool WIN>
// (Zo: the conditional's normaliser sigma_a + sigma_b, when it is computed)
__device__ __forceinline__ int32_t draw_token(const DevModel &M, const TokenIn &tk, DocState<CT, WIN> &S, const double *R,
                                              const int g, const int32_t side_ratio, ZCount &cnt, double &Zo)
{
    CT *mt = S.mt;
    // m^{-i}: remove the token from its document's counts.  (Every lane of
    // the group stores the same count to the same address: one store without
    // a lane mask, cheaper than the branch around a single lane's store.)
    const int32_t kold = tk.kold;
    const int32_t mo = mt[kold];
    __builtin_amdgcn_wave_barrier();
    mt[kold] = (CT)(mo - 1);
    __builtin_amdgcn_wave_barrier();
    const int32_t Kv = tk.kv;
    // (tested for the wave first: a wave without such a token skips the
    // lane-masked branch)
    if (__builtin_amdgcn_ballot_w64(Kv == 0) != 0 && Kv == 0) {
        // 0/0 conditional: the token keeps its topic
        mt[kold] = (CT)mo;
        __builtin_amdgcn_wave_barrier();
        cnt.degenerate++;
        return -1 - kold;
    }
    // the document's topics with a nonzero count besides the token
    const int32_t Kd = S.L - (mo == 1 ? 1 : 0);
    cnt.j += (uint32_t)(Kd < Kv ? Kd : Kv);
    // b-terms over one side: the document's topics (lst) or the word's Phi
    // column, ascending topic order either way.  The column is read
    // contiguously while the document side gathers single draws from the
    // dense column, so a group prefers the column side up to side_ratio
    // times the document's topic count.  The side is taken for the whole
    // wave (the document side if any of its groups prefers it: a frequent
    // word's column is long, a document's topic list is not), so the
    // wave's groups do not diverge; the side changes cost, not the law.
    int32_t knew = -1;
    // when every group's token in the wave takes the a-part whatever its
    // b-terms (decided at staging), the b-terms are not needed
    if (__builtin_amdgcn_ballot_w64(tk.sure == 0) != 0) {
        const bool prefer_doc = Kd == 0 || (uint32_t)Kv > __umul24((uint32_t)side_ratio, (uint32_t)Kd);
        const bool doc = __builtin_amdgcn_ballot_w64(prefer_doc) != 0;
        // terms per lane and round: a half or three quarters of the
        // registers' worth when no group of the wave has more than that many
        // per lane (one round either way)
        constexpr int KP = keep_of<G>();
        const int32_t J = doc ? S.L : Kv;
        const bool over2 = __builtin_amdgcn_ballot_w64(J > (KP / 2) * G) != 0;
        const bool over3 = __builtin_amdgcn_ballot_w64(J > (3 * KP / 4) * G) != 0;
        if (doc)
            knew = !over2 ? b_part<G, true, CT, KP / 2>(M, tk, S, R, g, Zo)
                          : (!over3 ? b_part<G, true, CT, 3 * KP / 4>(M, tk, S, R, g, Zo)
                                    : b_part<G, true, CT, KP>(M, tk, S, R, g, Zo));
        else
            knew = !over2 ? b_part<G, false, CT, KP / 2>(M, tk, S, R, g, Zo)
                          : (!over3 ? b_part<G, false, CT, 3 * KP / 4>(M, tk, S, R, g, Zo)
                                    : b_part<G, false, CT, KP>(M, tk, S, R, g, Zo));
    }
    if (knew < 0) {
        // a-part: the word's alias table over alpha_k phi_kv (drawn when the
        // token was staged)
        knew = tk.ka;
        cnt.a++;
    }
    // add the token back with its new topic
    const int32_t mn = mt[knew];
    __builtin_amdgcn_wave_barrier();
    mt[knew] = (CT)(mn + 1);
    __builtin_amdgcn_wave_barrier();
    list_update<G>(S, kold, knew, mo, mn, g);
    return knew;
}

// the fp64 b-part for the draws the fp32 one leaves undecided (a few per
// ten thousand tokens), with the fields it reads in registers
template <int G, bool DOC, typename CT, int KP>
__device__ __forceinline__ int32_t b_part_fp64(uint32_t *ckg, uint16_t *g16, float *phid, const double *Rd,
                                               const double *sigma_a, const int32_t phi_method, const TokenZ tz,
                                               CT *mt, uint16_t *lst, const int32_t L, const int g)
{
    // the fields b_part reads, in registers
    DevModel M;
    M.ckg = ckg;
    M.g16 = g16;
    M.phid = phid;
    M.phi_method = phi_method;
    TokenIn tk;
    tk.vk = tz.vk;
    tk.cb = tz.cb;
    tk.kv = tz.kv;
    tk.u0 = tz.u0;
    tk.vs = tz.vs;
    tk.sa = sigma_a[tz.v];
    DocState<CT, true> S;
    S.mt = mt;
    S.lst = lst;
    S.L = L;
    double Zo;
    return b_part<G, DOC, CT, KP>(M, tk, S, Rd, g, Zo);
}

// draw_token with the b-part in fp32 (b_part_f32), the fp64 b_part for the
// draws it leaves undecided: the same results.  Rf (LDS) holds fp32(R_k);
// the fp64 path reads R_k from global memory.
// EARLY: each b-term round's LDS reads issued before its gathered draws are
// used (the z-step's choice; the fold-in kernel draws faster without)
template <int G, typename CT, bool WIN, bool EARLY = WIN>
__device__ __forceinline__ int32_t draw_token_f32(const DevModel &M, const TokenZ &tk, DocState<CT, WIN> &S,
                                                  const float *Rf, const int g, const int32_t side_ratio,
                                                  ZCount32 &cnt)
{
    CT *mt = S.mt;
    const int32_t kold = tk.kold;
    const int32_t mo = mt[kold];
    __builtin_amdgcn_wave_barrier();
    mt[kold] = (CT)(mo - 1);
    __builtin_amdgcn_wave_barrier();
    const int32_t Kv = tk.kv;
    if (__builtin_amdgcn_ballot_w64(Kv == 0) != 0 && Kv == 0) {
        mt[kold] = (CT)mo;
        __builtin_amdgcn_wave_barrier();
        cnt.deg++;
        return -1 - kold;
    }
    const int32_t Kd = S.L - (mo == 1 ? 1 : 0);
    const uint32_t jt = (uint32_t)(Kd < Kv ? Kd : Kv);
    cnt.j += jt;
    cnt.jb += tk.sure ? 0u : jt;
    int32_t knew = -1;
    if (__builtin_amdgcn_ballot_w64(tk.sure == 0) != 0) {
        const bool prefer_doc = Kd == 0 || (uint32_t)Kv > __umul24((uint32_t)side_ratio, (uint32_t)Kd);
        const bool doc = __builtin_amdgcn_ballot_w64(prefer_doc) != 0;
        constexpr int KP = keep_of<G>();
        const int32_t J = doc ? S.L : Kv;
        const bool over2 = __builtin_amdgcn_ballot_w64(J > (KP / 2) * G) != 0;
        const bool over3 = __builtin_amdgcn_ballot_w64(J > (3 * KP / 4) * G) != 0;
        if (doc)
            knew = !over2 ? b_part_f32<G, true, CT, KP / 2, WIN, EARLY>(M, tk, S, Rf, g)
                          : (!over3 ? b_part_f32<G, true, CT, 3 * KP / 4, WIN, EARLY>(M, tk, S, Rf, g)
                                    : b_part_f32<G, true, CT, KP, WIN, EARLY>(M, tk, S, Rf, g));
        else
            knew = !over2 ? b_part_f32<G, false, CT, KP / 2, WIN, EARLY>(M, tk, S, Rf, g)
                          : (!over3 ? b_part_f32<G, false, CT, 3 * KP / 4, WIN, EARLY>(M, tk, S, Rf, g)
                                    : b_part_f32<G, false, CT, KP, WIN, EARLY>(M, tk, S, Rf, g));
        if (__builtin_amdgcn_ballot_w64(knew == -2) != 0) {
            // a draw too close to a boundary for fp32: the fp64 b-part
            const int32_t k64 = doc ? b_part_fp64<G, true, CT, KP>(M.ckg, M.g16, M.phid, M.Rd, M.sigma_a,
                                                                   M.phi_method, tk, S.mt, S.lst, S.L, g)
                                    : b_part_fp64<G, false, CT, KP>(M.ckg, M.g16, M.phid, M.Rd, M.sigma_a,
                                                                    M.phi_method, tk, S.mt, S.lst, S.L, g);
            if (knew == -2) {
                knew = k64;
                cnt.fb++;
            }
        }
    }
    if (knew < 0) {
        knew = tk.ka;
        cnt.a++;
    }
    const int32_t mn = mt[knew];
    __builtin_amdgcn_wave_barrier();
    mt[knew] = (CT)(mn + 1);
    __builtin_amdgcn_wave_barrier();
    list_update<G>(S, kold, knew, mo, mn, g);
    return knew;
}

// a token whose a-part was decided at staging (tk.sure): the same count and
// list updates as draw_token, with the new topic the word's alias draw
template <int G, typename CT, bool WIN>
__device__ __forceinline__ int32_t move_token(const TokenZ &tk, DocState<CT, WIN> &S, const int g, ZCount32 &cnt)
{
    CT *mt = S.mt;
    const int32_t kold = tk.kold;
    const int32_t mo = mt[kold];
    __builtin_amdgcn_wave_barrier();
    mt[kold] = (CT)(mo - 1);
    __builtin_amdgcn_wave_barrier();
    const int32_t Kv = tk.kv;
    const int32_t Kd = S.L - (mo == 1 ? 1 : 0);
    cnt.j += (uint32_t)(Kd < Kv ? Kd : Kv);
    const int32_t knew = tk.ka;
    cnt.a++;
    const int32_t mn = mt[knew];
    __builtin_amdgcn_wave_barrier();
    mt[knew] = (CT)(mn + 1);
    __builtin_amdgcn_wave_barrier();
    list_update<G>(S, kold, knew, mo, mn, g);
    return knew;
}

// load a document's topic counts into the group's LDS table (CT: 8-bit
// counts for documents shorter than 256 tokens, else 16-bit) and list them
template <int G, typename CT, bool WIN>
__device__ __forceinline__ void load_doc_counts(DocState<CT, WIN> &S, const uint16_t *z, int64_t s, int64_t e, int g,
                                                int32_t K, int32_t m_words)
{
    constexpr int PER_WORD = 4 / sizeof(CT);   // counters per 32-bit word
    constexpr int SHIFT = 8 * sizeof(CT);
    uint32_t *w32 = (uint32_t *)S.mt;
    for (int32_t i = g; i < m_words; i += G) w32[i] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int64_t i = s + g; i < e; i += G) {
        const int32_t k = z[i];
        atomicAdd(w32 + k / PER_WORD, 1u << (SHIFT * (k % PER_WORD)));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    build_list<G, CT>(S, g, K);
}

// stage the inputs of tokens i0 + g (one per lane) for a block of draws.
// nd: tokens of the document (0: never decide the a-part here).  The b-terms
// of a token sum to sigma_b = sum_k phi_kv m_k <= phimax(v) (nd - 1), so when
// u (sigma_a + phimax(v) (nd - 1)) < sigma_a the token takes the a-part
// whatever the counts; the test keeps a margin of 2^-36 relative, far above
// the rounding of either side's sums, so it never decides a token that the
// full computation (or the definition's order of sums) would send to the
// b-part.
__device__ __forceinline__ void stage_token(const DevModel &M, TokenIn *tok, int g, int32_t v, int32_t kold,
                                            const r4 &r, const int32_t nd)
{
    TokenIn x;
    x.vk = (uint32_t)v * (uint32_t)M.K;
    x.vs = (uint32_t)v * (uint32_t)M.ks16;
    x.cb = M.colptr[v];
    x.kold = (uint16_t)kold;
    const int32_t kv = M.colptr[v + 1] - x.cb;
    x.kv = (uint16_t)kv;
    x.u0 = (float)(r.x >> 8) * 0x1p-24f;
    x.sa = M.sigma_a[v];
    // the a-part's draw from the word's alias table over alpha_k phi_kv:
    // slot j = floor(r1 * K_v / 2^32), kept when r2 < its threshold, else
    // its alias (Section 3.5)
    uint32_t ka = 0;
    if (kv > 0) {
        const uint32_t j = scale32(r.y, (uint32_t)kv);
        const uint64_t a = M.calias[x.cb + j];
        ka = (r.z < (uint32_t)a) ? (uint32_t)((a >> 32) & 0xFFFFu) : (uint32_t)(a >> 48);
    }
    x.ka = (uint16_t)ka;
    bool sure = false;
    if (kv > 0 && nd > 0) {
        const double B = (double)M.phimax[v] * (double)(nd - 1);
        sure = unit24(r.x) * (x.sa + B) < x.sa * (1.0 - 0x1p-36);
    }
    x.sure = sure ? 1 : 0;
    tok[g] = x;
}

// stage the inputs of the z-step's token at lane g from its word's record:
// as stage_token, with the a-part decided at staging by the same bound in
// fp32: u (sigma_a + phimax(v) (nd - 1)) < sigma_a (1 - 2^-20), both sides
// rounded to fp32 (a relative error below 6 2^-24 each), so a token so
// decided has x < sigma_a (1 - 10 2^-24) exactly, far outside any rounding
// of the sums (the fp64 and exact decisions agree)
// (returns the token's sure flag)
__device__ __forceinline__ bool stage_token_z(const DevModel &M, TokenZ *tok, int g, int32_t v, int32_t kold,
                                              const r4 &r, const int32_t nd)
{
    const uint4 rec = M.wrec[v];
    TokenZ x;
    x.vk = (uint32_t)v * (uint32_t)M.K;
    x.vs = (uint32_t)v * (uint32_t)M.ks16;
    x.cb = (int32_t)rec.x;
    x.kold = (uint16_t)kold;
    const uint32_t kv = rec.y;
    x.kv = (uint16_t)kv;
    x.u0 = (float)(r.x >> 8) * 0x1p-24f;
    x.saf = __uint_as_float(rec.z);
    x.v = (uint32_t)v;
    uint32_t ka = 0;
    if (kv > 0) {
        const uint32_t j = scale32(r.y, kv);
        const uint64_t a = M.calias[rec.x + j];
        ka = (r.z < (uint32_t)a) ? (uint32_t)((a >> 32) & 0xFFFFu) : (uint32_t)(a >> 48);
    }
    x.ka = (uint16_t)ka;
    bool sure = false;
    if (kv > 0 && nd > 0) {
        const float B = __uint_as_float(rec.w) * (float)(nd - 1);
        sure = x.u0 * (x.saf + B) < x.saf * (1.0f - 0x1p-20f);
    }
    x.sure = sure ? 1 : 0;
    tok[g] = x;
    return sure;
}

// HOT: the frequent words' count increments go to the block's counters in
// LDS (hist), the others' to n
template <int G, typename CT, bool HOT>
__device__ void z_step_item(const ZArgs &a, const WorkItem &w, const float *R, uint8_t *wave_base,
                            TokenZ *wave_tok, unsigned long long *wave_cnt, uint32_t *hist)
{
    constexpr int NG = 64 / G;
    const int lane = __lane_id();
    const int g = lane & (G - 1);
    const int grp = lane / G;
    DocState<CT, true> S;
    S.mt = (CT *)(wave_base + grp * a.group_bytes);
    S.lst = (uint16_t *)(wave_base + grp * a.group_bytes + a.m_bytes);
    TokenZ *tok = wave_tok + grp * G;
    const DevModel &M = a.m;
    const uint32_t t = *M.tptr;
    for (int32_t di = grp; di < w.count; di += NG) {
        const int32_t d = a.c.doc_order[w.first + di];
        const int64_t s = a.c.doc_off[d], e = a.c.doc_off[d + 1];
        if (s == e) {
            if (a.ll_doc && g == 0) a.ll_doc[d] = 0.0;
            continue;
        }
        load_doc_counts<G, CT>(S, a.c.z, s, e, g, M.K, a.m_bytes / 4);
        ZCount32 cnt = {0, 0, 0, 0, 0};
        for (int64_t i0 = s; i0 < e; i0 += G) {
            const int64_t i = i0 + g;
            const bool valid = i < e;
            int32_t zo = 0, wv = 0;
            bool sure = false;
            if (valid) {
                // the token stream is read once per sweep: non-temporal, so
                // it does not displace the tables the draws reuse
                wv = __builtin_nontemporal_load(a.c.words + i);
                zo = __builtin_nontemporal_load(a.c.z + i);
                const r4 r = philox((uint32_t)i, (uint32_t)((uint64_t)i >> 32), t, TAG_Z, M.key0, M.key1);
                sure = stage_token_z(M, tok, g, wv, zo, r, (int32_t)(e - s));
            }
            // bit j: the group's token j was decided at staging (the cursor
            // tests it in a register instead of reading LDS)
            const auto sure_bits = (typename std::conditional<(G > 32), uint64_t, uint32_t>::type)group_ballot<G>(sure);
            __builtin_amdgcn_wave_barrier();
            int32_t znew = zo;
            const int nb = (int)((e - i0) < G ? (e - i0) : G);
            // each group walks its tokens with its own cursor: the tokens
            // whose a-part was decided at staging move at once, then every
            // group with a token left draws it, all groups together, so a
            // wave runs the b-terms as often as its busiest group needs.
            // (With 8 groups a wave the runs of decided tokens no longer line
            // up: those groups draw in step, and skip the b-terms only when
            // all eight tokens are decided.)
            if constexpr (G < 16) {
                for (int jj = 0; jj < nb; ++jj) {
                    const TokenZ tk = tok[jj];
                    int32_t k = draw_token_f32<G, CT>(M, tk, S, R, g, w.side_ratio, cnt);
                    if (k < 0) k = -1 - k;
                    if (g == jj) znew = k;
                }
            } else {
            int cur = 0;
            while (true) {
                while (cur < nb && ((sure_bits >> cur) & 1u)) {
                    const TokenZ tk = tok[cur];
                    const int32_t k = move_token<G, CT>(tk, S, g, cnt);
                    if (g == cur) znew = k;
                    ++cur;
                }
                if (cur < nb) {
                    const TokenZ tk = tok[cur];
                    int32_t k = draw_token_f32<G, CT>(M, tk, S, R, g, w.side_ratio, cnt);
                    if (k < 0) k = -1 - k;
                    if (g == cur) znew = k;
                    ++cur;
                }
                if (__builtin_amdgcn_ballot_w64(cur < nb) == 0) break;
            }
            }
            __builtin_amdgcn_wave_barrier();
            // the count rebuild: each lane adds its own token, once the
            // block's draws are done (a frequent word's into the block's
            // counters in LDS, added to n when the kernel ends)
            if (valid) {
                __builtin_nontemporal_store((uint16_t)znew, a.c.z + i);
                const int32_t h = HOT ? M.hot[wv] : -1;
                if (HOT && h >= 0) atomicAdd(&hist[(uint32_t)h * (uint32_t)M.K + (uint32_t)znew], 1u);
                else atomicAdd(&M.n[(uint32_t)wv * (uint32_t)M.K + (uint32_t)znew], 1);
            }
        }
        if (g == 0) {
            atomicAdd(&wave_cnt[0], (unsigned long long)cnt.j);
            atomicAdd(&wave_cnt[1], (unsigned long long)cnt.a);
            atomicAdd(&wave_cnt[2], (unsigned long long)cnt.deg);
            atomicAdd(&wave_cnt[3], (unsigned long long)cnt.jb);
            atomicAdd(&wave_cnt[4], (unsigned long long)cnt.fb);
        }
        if (a.ll_doc) {
            // the document's term of log p(z | alpha) for its final counts:
            // lgamma(A) - lgamma(N_d + A) + sum_k [lgamma(m_k + alpha) - lgamma(alpha)]
            int32_t base;
            const int32_t n = list_block<G>(S.L, g, base);
            double part = 0.0;
            for (int32_t j = 0; j < n; ++j) part += M.lg_alpha[S.mt[S.lst[base + j]]];
            const double tot = group_bcast_f64<G>(group_scan_incl<G>(part), G - 1);
            if (g == 0) a.ll_doc[d] = tot + M.lg_A[e - s];
        }
    }
}

// one persistent kernel per group size and count width: waves take work
// items from this class's queue until it is empty
// 5 waves per SIMD (96 VGPRs): more resident groups hide the chains'
// latency, more than 96 registers would spill in the draw loop.  Groups of
// 8 keep 8 b-terms per lane and their LDS allows 2 waves per SIMD, so they
// take the registers instead.
template <int G, typename CT, bool HOT>
__global__ void __launch_bounds__(256, (G == 8 ? 2 : 5)) z_step_kernel(ZArgs a)
{
    extern __shared__ __align__(16) uint8_t z_lds[];
    // fp32(R_k) for the fp32 b-terms (the fp64 path reads R_k from global
    // memory)
    float *R = (float *)z_lds;
    for (int32_t k = threadIdx.x; k < a.m.K; k += blockDim.x) R[k] = (float)a.m.Rd[k];
    // the block's counters of the frequent words' increments
    uint32_t *hist = (uint32_t *)(z_lds + a.hot_off);
    const int32_t n_hist = HOT ? a.n_hot * a.m.K : 0;
    for (int32_t i = threadIdx.x; i < n_hist; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    uint8_t *blk = z_lds + a.r_bytes;
    uint8_t *wave_base = blk + wave * a.wave_bytes;
    TokenZ *wave_tok = (TokenZ *)(blk + 4 * a.wave_bytes) + wave * 64;
    // the wave's statistics: sum of J, a-part draws, degenerate tokens, sum
    // of J over the tokens whose b-terms were computed, fp64 fallbacks
    unsigned long long *wave_cnt = (unsigned long long *)(blk + 4 * a.wave_bytes + 4 * 64 * sizeof(TokenZ)) + 5 * wave;
    if (__lane_id() < 5) wave_cnt[__lane_id()] = 0ull;
    __builtin_amdgcn_wave_barrier();
    while (true) {
        int item = 0;
        if (__lane_id() == 0) item = atomicAdd(a.queue, 1);
        item = __builtin_amdgcn_readlane(item, 0);
        if (item >= a.n_items) break;
        // a private copy: a reference into global memory would be reloaded
        // after every store of the item (stores may alias it)
        const WorkItem w = a.items[item];
        z_step_item<G, CT, HOT>(a, w, R, wave_base, wave_tok, wave_cnt, hist);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (a.stats && __lane_id() < 5) {
        const unsigned long long v = wave_cnt[__lane_id()];
        const int l = __lane_id();
        const int idx = l == 0 ? ST_SUM_J : (l == 1 ? ST_SUM_A : (l == 2 ? ST_DEGENERATE : (l == 3 ? ST_SUM_JB : ST_FALLBACK)));
        if (v) atomicAdd(&a.stats[idx], v);
    }
    if (HOT) {
        // every wave of the block is done: add the block's counters to n
        __syncthreads();
        const int32_t K = a.m.K;
        for (int32_t i = threadIdx.x; i < n_hist; i += blockDim.x) {
            const uint32_t c = hist[i];
            const int32_t h = i / K;
            if (c) atomicAdd(&a.m.n[(uint32_t)a.m.hot_word[h] * (uint32_t)K + (uint32_t)(i - h * K)], (int32_t)c);
        }
    }
}

// ---------------------------------------------------------------------------
// z-step, one document per lane (documents shorter than 128 tokens).  Lane l
// keeps its document's topics with a nonzero count as an ascending list of
// (topic, count) in LDS, entry j at j*64 + l so that the lanes' j-th entries
// are adjacent.  A token's b-terms are summed over the whole list in
// ascending topic order, one after the other in the lane (a listed topic
// the word's column lacks adds a zero term), so the running sums are those
// of the definition term by term.  The running sum after every block of 8
// entries stays in registers; the b-part walk re-reads one block.
// ---------------------------------------------------------------------------
constexpr int LANE_CAP = 127;                                      // list capacity
constexpr int LANE_BLK = 8;                                        // entries per gather batch
constexpr int LANE_NBLK = (LANE_CAP + LANE_BLK - 1) / LANE_BLK;    // 16

// first index j of the lane's list with topic >= key
__device__ __forceinline__ int32_t lane_lower_bound(const uint16_t *kl, int32_t L, int32_t key)
{
    int32_t lo = 0, hi = L;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int32_t)kl[mid * 64] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// one block of the lane's list: b-terms of entries [j0, j0 + 8) (zero past L)
__device__ __forceinline__ void lane_block_terms(const uint16_t *kl, const uint8_t *ml, int32_t L, int32_t j0,
                                                 const uint16_t *g16col, const float *pcol, const double *Rd,
                                                 int32_t (&kk)[LANE_BLK], double (&bb)[LANE_BLK])
{
    uint32_t mm[LANE_BLK], xx[LANE_BLK];
    double rr[LANE_BLK];
#pragma unroll
    for (int u = 0; u < LANE_BLK; ++u) {
        const bool ok = j0 + u < L;
        const int32_t j = ok ? j0 + u : 0;
        const int32_t k = kl[j * 64];
        const uint32_t m = ml[j * 64];
        kk[u] = ok ? k : 0;
        mm[u] = ok ? m : 0u;
    }
#pragma unroll
    for (int u = 0; u < LANE_BLK; ++u) {
        xx[u] = g16col[(uint32_t)kk[u]];
        rr[u] = Rd[kk[u]];
    }
    // phi_kv = fp32(x * R_k) == fp32(RN64(x / S_k)); escapes (0xFFFF) read
    // the fp32 table
    float fk[LANE_BLK];
    bool esc = false;
#pragma unroll
    for (int u = 0; u < LANE_BLK; ++u) {
        fk[u] = (float)((double)xx[u] * rr[u]);
        esc |= xx[u] == 0xFFFFu;
    }
    if (__builtin_amdgcn_ballot_w64(esc)) {
#pragma unroll
        for (int u = 0; u < LANE_BLK; ++u)
            if (xx[u] == 0xFFFFu) fk[u] = pcol[kk[u]];
    }
#pragma unroll
    for (int u = 0; u < LANE_BLK; ++u) bb[u] = (double)fk[u] * (double)mm[u];
}

__global__ void __launch_bounds__(64) z_lane_kernel(ZArgs a)
{
    extern __shared__ __align__(16) uint8_t l_lds[];
    const int lane = __lane_id();
    uint16_t *kl = (uint16_t *)l_lds + lane;                            // entry j at kl[j * 64]
    uint8_t *ml = l_lds + LANE_CAP * 64 * sizeof(uint16_t) + lane;      // entry j at ml[j * 64]
    const DevModel &M = a.m;
    const uint32_t t = *M.tptr;
    ZCount cnt = {0, 0, 0, 0, 0};
    while (true) {
        int item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1);
        item = __builtin_amdgcn_readlane(item, 0);
        if (item >= a.n_items) break;
        const WorkItem w = a.items[item];
        for (int32_t di = lane; di < w.count; di += 64) {
            const int32_t d = a.c.doc_order[w.first + di];
            const int64_t s = a.c.doc_off[d], e = a.c.doc_off[d + 1];
            // the document's counts as an ascending (topic, count) list
            int32_t L = 0;
            for (int64_t i = s; i < e; ++i) {
                const int32_t k = a.c.z[i];
                const int32_t pos = lane_lower_bound(kl, L, k);
                if (pos < L && kl[pos * 64] == k) {
                    ml[pos * 64] += 1;
                } else {
                    for (int32_t j = L - 1; j >= pos; --j) {
                        kl[(j + 1) * 64] = kl[j * 64];
                        ml[(j + 1) * 64] = ml[j * 64];
                    }
                    kl[pos * 64] = (uint16_t)k;
                    ml[pos * 64] = 1;
                    ++L;
                }
            }
            for (int64_t i = s; i < e; ++i) {
                const int32_t v = a.c.words[i];
                const int32_t kold = a.c.z[i];
                const int32_t cb = M.colptr[v];
                const int32_t Kv = M.colptr[v + 1] - cb;
                int32_t knew = kold;
                if (Kv == 0) {
                    // 0/0 conditional: the token keeps its topic
                    cnt.degenerate++;
                } else {
                    const r4 r = philox((uint32_t)i, (uint32_t)((uint64_t)i >> 32), t, TAG_Z, M.key0, M.key1);
                    const double sa = M.sigma_a[v];
                    const uint64_t al = M.calias[cb + scale32(r.y, (uint32_t)Kv)];
                    const int32_t ka = (r.z < (uint32_t)al) ? (int32_t)((al >> 32) & 0xFFFFu) : (int32_t)(al >> 48);
                    // m^{-i}
                    const int32_t po = lane_lower_bound(kl, L, kold);
                    const int32_t mo = ml[po * 64];
                    ml[po * 64] = (uint8_t)(mo - 1);
                    const int32_t Kd = L - (mo == 1 ? 1 : 0);
                    cnt.J += (unsigned long long)(Kd < Kv ? Kd : Kv);
                    const uint16_t *g16col = M.g16 + (uint32_t)v * (uint32_t)M.ks16;
                    const float *pcol = M.phid + (uint32_t)v * (uint32_t)M.K;
                    // sigma_b over the list, ascending, with the running sum after each block
                    double bs[LANE_NBLK];
                    double sb = 0.0;
                    int32_t last = -1;
    #pragma unroll
                    for (int blk = 0; blk < LANE_NBLK; ++blk) {
                        bs[blk] = sb;
                        if (!__builtin_amdgcn_ballot_w64(blk * LANE_BLK < L)) continue;
                        int32_t kk[LANE_BLK];
                        double bb[LANE_BLK];
                        lane_block_terms(kl, ml, L, blk * LANE_BLK, g16col, pcol, M.Rd, kk, bb);
    #pragma unroll
                        for (int u = 0; u < LANE_BLK; ++u) {
                            sb += bb[u];
                            if (bb[u] > 0.0) last = blk * LANE_BLK + u;
                        }
                        bs[blk] = sb;
                    }
                    const double x = unit24(r.x) * (sa + sb);
                    if (x < sa) {
                        knew = ka;
                        cnt.A++;
                    } else {
                        // b-part: the block whose running sum first passes y, then its entries
                        const double y = x - sa;
                        int32_t blk = -1;
                        double c0 = 0.0;
    #pragma unroll
                        for (int b = LANE_NBLK - 1; b >= 0; --b) {
                            if (bs[b] > y) {
                                blk = b;
                                c0 = b > 0 ? bs[b - 1] : 0.0;
                            }
                        }
                        knew = -1;
                        if (blk >= 0) {
                            int32_t kk[LANE_BLK];
                            double bb[LANE_BLK];
                            lane_block_terms(kl, ml, L, blk * LANE_BLK, g16col, pcol, M.Rd, kk, bb);
                            double c = c0;
    #pragma unroll
                            for (int u = 0; u < LANE_BLK; ++u) {
                                c += bb[u];
                                if (knew < 0 && bb[u] > 0.0 && c > y) knew = kk[u];
                            }
                        }
                        // no running sum passed y (rounding): the last positive term
                        if (knew < 0) knew = kl[last * 64];
                    }
                    // counts and list
                    if (knew == kold) {
                        ml[po * 64] = (uint8_t)mo;
                    } else {
                        if (mo == 1) {
                            for (int32_t j = po; j < L - 1; ++j) {
                                kl[j * 64] = kl[(j + 1) * 64];
                                ml[j * 64] = ml[(j + 1) * 64];
                            }
                            --L;
                        }
                        const int32_t pn = lane_lower_bound(kl, L, knew);
                        if (pn < L && kl[pn * 64] == knew) {
                            ml[pn * 64] += 1;
                        } else {
                            for (int32_t j = L - 1; j >= pn; --j) {
                                kl[(j + 1) * 64] = kl[j * 64];
                                ml[(j + 1) * 64] = ml[j * 64];
                            }
                            kl[pn * 64] = (uint16_t)knew;
                            ml[pn * 64] = 1;
                            ++L;
                        }
                    }
                    a.c.z[i] = (uint16_t)knew;
                }
                atomicAdd(&M.n[(uint32_t)v * (uint32_t)M.K + (uint32_t)knew], 1);
            }
            if (a.ll_doc) {
                // lgamma(A) - lgamma(N_d + A) + sum_k [lgamma(m_k + alpha) - lgamma(alpha)]
                double part = 0.0;
                for (int32_t j = 0; j < L; ++j) part += M.lg_alpha[ml[j * 64]];
                a.ll_doc[d] = part + M.lg_A[e - s];
            }
        }
    }
    if (a.stats) {
        if (cnt.J) {
            atomicAdd(&a.stats[ST_SUM_J], (unsigned long long)cnt.J);
            atomicAdd(&a.stats[ST_SUM_JB], (unsigned long long)cnt.J);
        }
        if (cnt.A) atomicAdd(&a.stats[ST_SUM_A], (unsigned long long)cnt.A);
        if (cnt.degenerate) atomicAdd(&a.stats[ST_DEGENERATE], (unsigned long long)cnt.degenerate);
    }
}

static int ilog2(int x)
{
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

static int topics_per_lane_log2(int K, int G)
{
    int c = ilog2((K + G - 1) / G);
    return c;
}

__global__ void bump_kernel(unsigned long long *x)
{
    if (threadIdx.x == 0) *x += 1ull;
}

hipError_t launch_z_prepare(const DevModel &m, int32_t *queues, unsigned long long *stats, hipStream_t s)
{
    hipError_t e;
    if (m.n) {
        e = launch_fill_u32((uint32_t *)m.n, 0u, (int64_t)m.V * m.K, s);
        if (e != hipSuccess) return e;
    }
    if (stats) {
        bump_kernel<<<1, 64, 0, s>>>(&stats[ST_TOKENS]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_fill_u32((uint32_t *)queues, 0u, Z_QUEUES, s);
}

hipError_t launch_z_class(const DevCorpus &c, const DevModel &m, int32_t group, bool narrow, const WorkItem *items,
                          int32_t n_items, int32_t n_cu, int32_t *queue, unsigned long long *stats,
                          double *ll_doc, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if ((group == 8 || group == 1) && !narrow) return hipErrorInvalidValue;
    ZArgs a;
    a.m = m;
    a.c = c;
    a.items = items;
    a.n_items = n_items;
    a.queue = queue;
    a.stats = stats;
    a.ll_doc = m.lg_alpha ? ll_doc : nullptr;
    const ZLayout L = z_layout(group, narrow, m.K);
    a.m_bytes = L.m_bytes;
    a.group_bytes = L.group_bytes;
    a.wave_bytes = L.wave_bytes;
    a.r_bytes = L.r_bytes;
    size_t lds = ((size_t)a.r_bytes + 4 * ((size_t)a.wave_bytes + 64 * sizeof(TokenIn) + 40) + 15) / 16 * 16;
    a.n_hot = 0;
    a.hot_off = (int32_t)lds;
    auto launch = [&](auto kernel, auto kernel_hot) -> hipError_t {
        // persistent: exactly the blocks the device holds at once, and no
        // more waves than work items (a wave takes one item at a time)
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds);
        if (e != hipSuccess) return e;
        bool hot = false;
        if (m.n_hot > 0) {
            // the frequent words' counters in LDS, unless they cost blocks
            const size_t with = lds + (size_t)m.n_hot * m.K * 4;
            int per_cu_hot = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_hot, kernel_hot, 256, with);
            if (e != hipSuccess) return e;
            if (per_cu_hot == per_cu) {
                a.n_hot = m.n_hot;
                lds = with;
                hot = true;
            }
        }
        if (per_cu <= 0) return hipErrorInvalidConfiguration;  // the block's LDS exceeds the CU's
        int64_t blocks = (int64_t)per_cu * (n_cu > 0 ? n_cu : 1);
        const int64_t need = ((int64_t)n_items + 3) / 4;
        if (blocks > need) blocks = need;
        if (hot) kernel_hot<<<(unsigned)blocks, 256, lds, s>>>(a);
        else kernel<<<(unsigned)blocks, 256, lds, s>>>(a);
        return hipGetLastError();
    };
    if (group == 1) {
        // one document per lane: 64-thread blocks, the lanes' topic lists
        const size_t llds = (size_t)LANE_CAP * 64 * 3;
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, z_lane_kernel, 64, llds);
        if (e != hipSuccess) return e;
        if (per_cu <= 0) return hipErrorInvalidConfiguration;
        int64_t blocks = (int64_t)per_cu * (n_cu > 0 ? n_cu : 1);
        if (blocks > n_items) blocks = n_items;
        z_lane_kernel<<<(unsigned)blocks, 64, llds, s>>>(a);
        return hipGetLastError();
    }
    if (narrow) {
        if (group == 32) return launch(z_step_kernel<32, uint8_t, false>, z_step_kernel<32, uint8_t, true>);
        if (group == 16) return launch(z_step_kernel<16, uint8_t, false>, z_step_kernel<16, uint8_t, true>);
        return launch(z_step_kernel<8, uint8_t, false>, z_step_kernel<8, uint8_t, true>);
    }
    if (group == 64) return launch(z_step_kernel<64, uint16_t, false>, z_step_kernel<64, uint16_t, true>);
    if (group == 32) return launch(z_step_kernel<32, uint16_t, false>, z_step_kernel<32, uint16_t, true>);
    return launch(z_step_kernel<16, uint16_t, false>, z_step_kernel<16, uint16_t, true>);
}

// ---------------------------------------------------------------------------
// Collapsed log joint (Section 4 reports it per iteration):
//   words: K lgamma(V beta) - sum_k lgamma(n_k + V beta)
//          + sum_{k,v: n_kv > 0} [lgamma(n_kv + beta) - lgamma(beta)]
//   docs:  sum_d [lgamma(A) - lgamma(N_d + A)
//          + sum_{k: m_dk > 0} (lgamma(m_dk + alpha_k) - lgamma(alpha_k))]
// Partial sums per block in a fixed order, then one fixed-order reduction,
// so the value is the same on every run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_f64(double x, double *red)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) t += red[wv];
    return t;
}

// (beta_v: per-word priors, cells word-major with K per word; else the
// symmetric beta through the table of lgamma(x + beta) - lgamma(beta))
__global__ void __launch_bounds__(256) ll_words_kernel(const int32_t *n, int64_t cells, int32_t K, double beta,
                                                       double lgb, const double *lg_beta, const double *beta_v,
                                                       double *partials)
{
    __shared__ double red[4];
    double acc = 0.0;
    // lgamma(n + beta) - lgamma(beta) of one cell (zero for an empty cell)
    auto term = [&](int32_t c, int64_t i) -> double {
        if (c <= 0) return 0.0;
        if (beta_v) {
            const double b = beta_v[i / K];
            return lgamma((double)c + b) - lgamma(b);
        }
        return c < LG_TABLE ? lg_beta[c] : lgamma((double)c + beta) - lgb;
    };
    // four cells per 16-byte load (the table is 256-byte aligned), four
    // loads in flight per thread; the cells past a multiple of four after
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = cells >> 2;
    const int4 *q = (const int4 *)n;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        int4 a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = q[i + j * stride];
        for (int j = 0; j < 4; ++j) {
            const int64_t c0 = 4 * (i + j * stride);
            acc += term(a[j].x, c0) + term(a[j].y, c0 + 1) + term(a[j].z, c0 + 2) + term(a[j].w, c0 + 3);
        }
    }
    for (; i < n4; i += stride) {
        const int4 a = q[i];
        acc += term(a.x, 4 * i) + term(a.y, 4 * i + 1) + term(a.z, 4 * i + 2) + term(a.w, 4 * i + 3);
    }
    for (int64_t r = 4 * n4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < cells; r += stride)
        acc += term(n[r], r);
    const double t = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <bool SYM>
__global__ void __launch_bounds__(256) ll_docs_kernel(DevCorpus c, int32_t K, const double *alpha,
                                                      const double *lg_alpha, const double *lg_A, int32_t log2c,
                                                      double *partials)
{
    extern __shared__ uint16_t ll_lds[];
    __shared__ double red[4];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int32_t C = 1 << log2c;
    uint16_t *mt = ll_lds + wv * (64 * C);
    uint32_t *w32 = (uint32_t *)mt;
    double acc = 0.0;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t d = blockIdx.x * 4 + wv; d < c.D; d += nw) {
        const int64_t s = c.doc_off[d], e = c.doc_off[d + 1];
        for (int32_t i = lane; i < 32 * C; i += 64) w32[i] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int64_t i = s + lane; i < e; i += 64) {
            const int32_t k = c.z[i];
            const int32_t slot = (k & (C - 1)) * 64 + (k >> log2c);
            atomicAdd(w32 + (slot >> 1), (slot & 1) ? 65536u : 1u);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        double part = 0.0;
        for (int32_t b = 0; b < C; ++b) {
            const int32_t cnt = mt[b * 64 + lane];
            if (cnt) {
                const int32_t k = lane * C + b;
                if constexpr (SYM) part += lg_alpha[cnt];
                else part += lgamma((double)cnt + alpha[k]) - lgamma(alpha[k]);
            }
        }
        if (lane == 0) part += lg_A[e - s];
        acc += part;
    }
    const double t = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// fixed-order partial sums of the per-document terms written by the z-step
__global__ void __launch_bounds__(256) ll_docsum_kernel(const double *ll_doc, int64_t D, double *partials)
{
    __shared__ double red[4];
    const int64_t per = (D + gridDim.x - 1) / gridDim.x;
    const int64_t a = blockIdx.x * per, b = a + per < D ? a + per : D;
    double acc = 0.0;
    for (int64_t d = a + threadIdx.x; d < b; d += blockDim.x) acc += ll_doc[d];
    const double t = block_sum_f64(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// one block of 256: the topics' terms and the partial sums strided over the
// threads, then a fixed-order block sum (deterministic)
__global__ void __launch_bounds__(256) ll_final_kernel(const double *partials, int32_t np,
                                                       const unsigned long long *nk, int32_t K, double Vbeta,
                                                       double *out, double *hist, const uint32_t *hist_idx)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int32_t k = threadIdx.x; k < K; k += blockDim.x) acc -= lgamma((double)nk[k] + Vbeta);
    for (int32_t i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
    const double t = block_sum_f64(acc, red);
    if (threadIdx.x == 0) {
        const double ll = (double)K * lgamma(Vbeta) + t;
        *out = ll;
        if (hist) hist[*hist_idx] = ll;
    }
}

__global__ void advance_kernel(uint32_t *tptr, uint32_t *hist_idx)
{
    if (threadIdx.x == 0) {
        *tptr += 1u;
        *hist_idx += 1u;
    }
}

hipError_t launch_advance(uint32_t *tptr, uint32_t *hist_idx, hipStream_t s)
{
    advance_kernel<<<1, 64, 0, s>>>(tptr, hist_idx);
    return hipGetLastError();
}

hipError_t launch_loglik(const DevCorpus &c, const DevModel &m, double *partials, int32_t n_part_words,
                         int32_t n_part_docs, const double *ll_doc, double *out, double *hist,
                         const uint32_t *hist_idx, hipStream_t s)
{
    hipError_t e = launch_row_sums(m.n, m.V, m.K, m.nk, s);
    if (e != hipSuccess) return e;
    ll_words_kernel<<<n_part_words, 256, 0, s>>>(m.n, (int64_t)m.V * m.K, m.K, m.beta, lgamma(m.beta), m.lg_beta,
                                                 m.beta_v, partials);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ll_doc) {
        ll_docsum_kernel<<<n_part_docs, 256, 0, s>>>(ll_doc, c.D, partials + n_part_words);
    } else {
        const int log2c = topics_per_lane_log2(m.K, 64);
        const size_t lds = 4 * 64 * (1 << log2c) * sizeof(uint16_t);
        if (m.lg_alpha)
            ll_docs_kernel<true><<<n_part_docs, 256, lds, s>>>(c, m.K, m.alpha, m.lg_alpha, m.lg_A, log2c,
                                                               partials + n_part_words);
        else
            ll_docs_kernel<false><<<n_part_docs, 256, lds, s>>>(c, m.K, m.alpha, m.lg_alpha, m.lg_A, log2c,
                                                                partials + n_part_words);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ll_final_kernel<<<1, 256, 0, s>>>(partials, n_part_words + n_part_docs, m.nk, m.K, m.beta_sum, out, hist,
                                      hist_idx);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phi export / import (parity tests; serving models built elsewhere)
// ---------------------------------------------------------------------------
__global__ void export_phi_kernel(DevModel m, int64_t *colptr64, uint16_t *topic, int32_t *gam_e, float *phi_e,
                                  uint32_t *thr, uint16_t *alias_topic)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= m.V) return;
    const int lane = __lane_id();
    const int32_t a = m.colptr[v], b = m.colptr[v + 1];
    if (lane == 0) {
        colptr64[v] = a;
        if (v == m.V - 1) colptr64[m.V] = b;
    }
    for (int32_t e = a + lane; e < b; e += 64) {
        const int32_t k = m.ctopic[e];
        topic[e] = (uint16_t)k;
        phi_e[e] = m.cphi[e];
        gam_e[e] = m.phi_method == 1 ? 0 : m.gam[(int64_t)v * m.K + k];
        const uint64_t al = m.calias[e];
        thr[e] = (uint32_t)al;
        alias_topic[e] = (uint16_t)(al >> 48);
    }
}

hipError_t launch_export_phi(const DevModel &m, int64_t *colptr64, uint16_t *topic, int32_t *gam_e, float *phi_e,
                             uint32_t *thr, uint16_t *alias_topic, hipStream_t s)
{
    export_phi_kernel<<<(m.V + 3) / 4, 256, 0, s>>>(m, colptr64, topic, gam_e, phi_e, thr, alias_topic);
    return hipGetLastError();
}

__global__ void import_phi_kernel(DevModel m, const int64_t *colptr64, const uint16_t *topic, const float *phi_e,
                                  const uint32_t *thr, const uint16_t *alias_topic)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= m.V) return;
    const int lane = __lane_id();
    const int64_t a = colptr64[v], b = colptr64[v + 1];
    if (lane == 0) {
        m.colptr[v] = (int32_t)a;
        if (v == m.V - 1) m.colptr[m.V] = (int32_t)b;
    }
    float *pcol = m.phid + (int64_t)v * m.K;
    uint16_t *g16col = m.g16 + (int64_t)v * m.ks16;
    for (int32_t k = lane; k < m.K; k += 64) pcol[k] = 0.0f;
    for (int32_t k = lane; k < m.ks16; k += 64) g16col[k] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // values without draws behind them: every nonzero cell is read from phid
    float fmax = 0.0f;
    for (int64_t e = a + lane; e < b; e += 64) {
        const int32_t k = topic[e];
        fmax = phi_e[e] > fmax ? phi_e[e] : fmax;
        m.ctopic[e] = (uint16_t)k;
        m.cphi[e] = phi_e[e];
        m.ckg[e] = (uint32_t)k | (0xFFFFu << 16);
        pcol[k] = phi_e[e];
        g16col[k] = 0xFFFF;
        m.calias[e] = (uint64_t)thr[e] | ((uint64_t)k << 32) | ((uint64_t)alias_topic[e] << 48);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const float y = __shfl_xor(fmax, o, 64);
        fmax = y > fmax ? y : fmax;
    }
    if (lane == 0) m.phimax[v] = fmax;
}

hipError_t launch_import_phi(const DevModel &m, const int64_t *colptr64, const uint16_t *topic, const float *phi_e,
                             const uint32_t *thr, const uint16_t *alias_topic, hipStream_t s)
{
    import_phi_kernel<<<(m.V + 3) / 4, 256, 0, s>>>(m, colptr64, topic, phi_e, thr, alias_topic);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// counts export: n as CSC by word (ascending topic), m as CSR by document
// ---------------------------------------------------------------------------
__global__ void n_colcount_kernel(const int32_t *n, int32_t V, int32_t K, int64_t *cnt)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= V) return;
    const int lane = __lane_id();
    int32_t c = 0;
    for (int32_t k = lane; k < K; k += 64) c += n[(int64_t)v * K + k] > 0;
    c = group_scan_incl_i32<64>(c);
    if (lane == 63) cnt[v] = c;
}

__global__ void n_fill_kernel(const int32_t *n, int32_t V, int32_t K, const int64_t *colptr, uint16_t *topic,
                              int32_t *cnt)
{
    const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= V) return;
    const int lane = __lane_id();
    int64_t run = colptr[v];
    for (int32_t k0 = 0; k0 < K; k0 += 64) {
        const int32_t k = k0 + lane;
        const int32_t x = k < K ? n[(int64_t)v * K + k] : 0;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(x > 0);
        if (x > 0) {
            const int64_t e = run + __builtin_popcountll(bal & ((1ull << lane) - 1ull));
            topic[e] = (uint16_t)k;
            cnt[e] = x;
        }
        run += __builtin_popcountll(bal);
    }
}

hipError_t launch_counts_csc(const DevModel &m, const int64_t *colptr64, uint16_t *topic, int32_t *cnt,
                             int32_t *unused, hipStream_t s)
{
    (void)unused;
    n_fill_kernel<<<(m.V + 3) / 4, 256, 0, s>>>(m.n, m.V, m.K, colptr64, topic, cnt);
    return hipGetLastError();
}

// pass 0: per-column / per-document nonzero counts (int64) into rowcnt
// pass 1: fill CSR m with rowptr = rowcnt (already scanned)
__global__ void m_rows_kernel(DevCorpus c, int32_t K, int32_t log2c, int64_t *rowcnt_or_ptr, uint16_t *topic,
                              int32_t *cnt, int pass)
{
    extern __shared__ uint16_t m_lds[];
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    const int32_t C = 1 << log2c;
    uint16_t *mt = m_lds + wv * (64 * C);
    const int64_t d = blockIdx.x * 4 + wv;
    if (d >= c.D) return;
    const int64_t s = c.doc_off[d], e = c.doc_off[d + 1];
    for (int32_t i = lane; i < 64 * C; i += 64) mt[i] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int64_t i = s + lane; i < e; i += 64) {
        const int32_t k = c.z[i];
        const int32_t slot = (k & (C - 1)) * 64 + (k >> log2c);
        atomicAdd((uint32_t *)(mt + (slot & ~1)), (slot & 1) ? 65536u : 1u);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    int32_t mine = 0;
    for (int32_t b = 0; b < C; ++b) mine += mt[b * 64 + lane] > 0;
    const int32_t incl = group_scan_incl_i32<64>(mine);
    if (pass == 0) {
        if (lane == 63) rowcnt_or_ptr[d] = incl;
        return;
    }
    int64_t o = rowcnt_or_ptr[d] + incl - mine;
    for (int32_t b = 0; b < C; ++b) {
        const int32_t x = mt[b * 64 + lane];
        if (x > 0) {
            topic[o] = (uint16_t)(lane * C + b);
            cnt[o] = x;
            ++o;
        }
    }
}

hipError_t launch_counts_m(const DevCorpus &c, int32_t K, int64_t *rowcnt_or_ptr, uint16_t *topic, int32_t *cnt,
                           int pass, hipStream_t s)
{
    if (c.D == 0) return hipSuccess;
    const int log2c = topics_per_lane_log2(K, 64);
    m_rows_kernel<<<(unsigned)((c.D + 3) / 4), 256, 4 * 64 * (1 << log2c) * sizeof(uint16_t), s>>>(
        c, K, log2c, rowcnt_or_ptr, topic, cnt, pass);
    return hipGetLastError();
}

hipError_t launch_n_colcount(const DevModel &m, int64_t *cnt, hipStream_t s)
{
    n_colcount_kernel<<<(m.V + 3) / 4, 256, 0, s>>>(m.n, m.V, m.K, cnt);
    return hipGetLastError();
}

hipError_t launch_scan_i64(const int64_t *in, int64_t *out_excl, int64_t n, long long *scratch, hipStream_t s)
{
    return scan_excl<int64_t, int64_t>(in, out_excl, n, scratch, scratch + (n + SCAN_BLOCK - 1) / SCAN_BLOCK, s);
}

// ---------------------------------------------------------------------------
// Fold-in (Phi fixed, no count rebuild): each group owns one request slot.
// On its first step a slot drops tokens whose word is out of range or has an
// empty Phi column, and draws initial topics.  Every step then runs up to
// `budget` token draws, resuming where the previous step stopped (sweep and
// token within it, kept on the device), with counters (p, request, sweep):
// the draws do not depend on how a request's work is cut into steps.  The
// topic counts are accumulated after each sweep past the burn-in, and the
// step that ends the last sweep writes theta and the log-likelihood of the
// final state.
// ---------------------------------------------------------------------------
template <int G, bool SYM>
__device__ void foldin_slot(const DevModel &M, const DevFoldin &F, int32_t sid, const float *Rf, uint16_t *mt,
                            TokenZ *tok)
{
    // the count table (K u16, rounded to 16 bytes), then the topic list with
    // room for its windows (launch_foldin_step sizes the same layout)
    const int32_t Kp = (M.K + 7) & ~7;
    DocState<uint16_t, true> S;
    S.mt = mt;
    S.lst = mt + Kp;
    const int lane = __lane_id();
    const int g = lane & (G - 1);
    const int32_t K = M.K;
    const FoldSlot sl = F.slots[sid];
    int32_t *wds = F.words + sl.arena_off;
    int32_t *pos = F.pos + sl.arena_off;
    uint16_t *zz = F.z + sl.arena_off;
    uint32_t *acc = F.acc + (int64_t)sid * K;
    int32_t kept = 0, done = 0, next = 0;
    if (sl.fresh) {
        // drop tokens, compact the kept positions, draw initial topics
        int32_t run = 0;
        for (int32_t p0 = 0; p0 < sl.len; p0 += G) {
            const int32_t p = p0 + g;
            bool keep = false;
            if (p < sl.len) {
                const int32_t v = wds[p];
                keep = v >= 0 && v < M.V && M.colptr[v + 1] > M.colptr[v];
            }
            const uint64_t bal = group_ballot<G>(keep);
            if (keep) {
                const int32_t q = run + __builtin_popcountll(bal & ((1ull << g) - 1ull));
                pos[q] = p;
                const r4 r = philox((uint32_t)p, sl.req, 0u, TAG_FOLDIN_INIT, F.key0, F.key1);
                zz[q] = (uint16_t)scale32(r.x, (uint32_t)K);
            }
            run += __builtin_popcountll(bal);
        }
        kept = run;
        for (int32_t k = g; k < K; k += G) acc[k] = 0;
        if (g == 0) {
            F.kept[2 * sid] = kept;
            F.kept[2 * sid + 1] = sl.len - kept;
            F.fin[sid] = 0;
        }
        __threadfence();
    } else {
        kept = F.kept[2 * sid];
        done = F.prog[2 * sid];
        next = F.prog[2 * sid + 1];
        // finished in an earlier step (a step launched before the host
        // collected it): its results stay as they are
        if (done >= F.sweeps) return;
    }
    load_doc_counts<G, uint16_t>(S, zz, 0, kept, g, K, Kp / 2);
    ZCount32 st = {0, 0, 0, 0, 0};
    int32_t budget = sl.budget;
    while (budget > 0 && done < F.sweeps) {
        const int32_t s = done + 1;
        const int32_t t1 = kept - next < budget ? kept : next + budget;
        for (int32_t q0 = next; q0 < t1; q0 += G) {
            const int32_t q = q0 + g;
            const bool valid = q < t1;
            int32_t zo = 0;
            if (valid) {
                const int32_t p = pos[q];
                zo = zz[q];
                const r4 r = philox((uint32_t)p, sl.req, (uint32_t)s, TAG_FOLDIN_Z, F.key0, F.key1);
                stage_token_z(M, tok, g, wds[p], zo, r, kept);
            }
            __builtin_amdgcn_wave_barrier();
            int32_t znew = zo;
            const int nb = (t1 - q0) < G ? (t1 - q0) : G;
            // the z-step's draw: b-terms in fp32 where a rounding bound proves
            // the decision, the fp64 b-part elsewhere (the same results)
            for (int jj = 0; jj < nb; ++jj) {
                const TokenZ tk = tok[jj];
                int32_t k = draw_token_f32<G, uint16_t, true, false>(M, tk, S, Rf, g, 1, st);
                if (k < 0) k = -1 - k;
                if (g == jj) znew = k;
            }
            __builtin_amdgcn_wave_barrier();
            if (valid) zz[q] = (uint16_t)znew;
        }
        budget -= t1 - next;
        next = t1;
        if (next == kept) {
            // the sweep is complete
            if (s > F.burn_in) {
                for (int32_t k = g; k < K; k += G) acc[k] += mt[k];
            }
            done = s;
            next = 0;
        }
    }
    if (g == 0) {
        F.prog[2 * sid] = done;
        F.prog[2 * sid + 1] = next;
    }
    __threadfence();
    if (done == F.sweeps) {
        const double denom = (double)kept + F.A;
        const double ns = (double)(F.sweeps - F.burn_in);
        for (int32_t k = g; k < K; k += G)
            F.theta[(int64_t)sid * K + k] = (float)(((double)acc[k] / ns + M.alpha[k]) / denom);
        double part = 0.0;
        for (int32_t q = g; q < kept; q += G) part += log((double)M.phid[(int64_t)wds[pos[q]] * K + zz[q]]);
        for (int32_t k = g; k < K; k += G) {
            const int32_t c = mt[k];
            if (c > 0) {
                if constexpr (SYM) part += M.lg_alpha[c];
                else part += lgamma((double)c + M.alpha[k]) - lgamma(M.alpha[k]);
            }
        }
        const double tot = group_bcast_f64<G>(group_scan_incl<G>(part), G - 1);
        if (g == 0) F.ll[sid] = tot + M.lg_A[kept];
        // the step number last, once theta and ll are written (the group is
        // one wave: the fence orders every lane's writes before it)
        __threadfence();
        if (g == 0) F.fin[sid] = F.step_no;
    }
}

template <int G, bool SYM>
__global__ void __launch_bounds__(256) foldin_step_kernel(DevModel M, DevFoldin F, const int32_t *active,
                                                          int32_t n_active, int32_t per_group)
{
    extern __shared__ __align__(16) uint16_t f_lds[];
    // the block's copy of fp32(R_k), then the groups' tables, then staged
    // tokens
    float *R = (float *)f_lds;
    for (int32_t k = threadIdx.x; k < M.K; k += blockDim.x) R[k] = (float)M.Rd[k];
    __syncthreads();
    uint16_t *blk = f_lds + (M.K * 4 + 15) / 16 * 8;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    constexpr int gsz = G;
    const int grp = lane / gsz;
    const int ngw = 64 / gsz;
    const int64_t gid = ((int64_t)blockIdx.x * 4 + wave) * ngw + grp;
    uint16_t *mt = blk + (wave * ngw + grp) * per_group;
    TokenZ *tok = (TokenZ *)(blk + 4 * ngw * per_group) + wave * 64 + grp * gsz;
    if (gid >= n_active) return;
    const int32_t sid = active[gid];
    foldin_slot<G, SYM>(M, F, sid, R, mt, tok);
}

hipError_t launch_foldin_step(const DevModel &m, const DevFoldin &f, const int32_t *active, int32_t n_active,
                              hipStream_t s)
{
    if (n_active == 0) return hipSuccess;
    // per group (u16 units): the count table (K entries), then the topic
    // list (K entries, at least W slots a lane and W more for its windows),
    // each rounded to 16 bytes
    const int32_t W = f.group == 16 ? 8 : 4;   // the list's window (slots per lane)
    const int32_t lcap = m.K > W * f.group + W ? m.K : W * f.group + W;
    const int per_group = ((m.K + 7) & ~7) + ((lcap + 7) & ~7);
    const int ngw = 64 / f.group;
    const int64_t waves = (n_active + ngw - 1) / ngw;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const size_t lds = (size_t)(m.K * 4 + 15) / 16 * 16 + 4 * ngw * per_group * sizeof(uint16_t) +
                       4 * 64 * sizeof(TokenZ);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, foldin_step_kernel<64, true>, 256, lds);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) return hipErrorInvalidConfiguration;  // the block's LDS exceeds the CU's
#define PULDA_FOLDIN(G_, S_) foldin_step_kernel<G_, S_><<<blocks, 256, lds, s>>>(m, f, active, n_active, per_group)
    if (m.lg_alpha) {
        if (f.group == 64) PULDA_FOLDIN(64, true);
        else if (f.group == 32) PULDA_FOLDIN(32, true);
        else PULDA_FOLDIN(16, true);
    } else {
        if (f.group == 64) PULDA_FOLDIN(64, false);
        else if (f.group == 32) PULDA_FOLDIN(32, false);
        else PULDA_FOLDIN(16, false);
    }
#undef PULDA_FOLDIN
    return hipGetLastError();
}



// ---------------------------------------------------------------------------
// Held-out log-likelihood of new documents, log p(w_d | Phi, alpha), by the
// left-to-right algorithm of Wallach, Murray, Salakhutdinov and Mimno, the
// estimator behind the held-out comparison of Section 4.  One group of G
// lanes per (document, particle).  Tokens whose word is >= V or whose Phi
// column is empty are dropped; at step n (n = 0 .. nk - 1) the particle
// redraws its topics z_0 .. z_{n-1} in order, each from the token
// conditional of Section 3.5 given its other topics among the first n (the
// fold-in draw), then draws z_n from that conditional given z_<n and keeps
// its normaliser Z_n = sigma_a(w_n) + sigma_b(w_n).  A second kernel forms
// sum_n log((1/R) sum_r Z_n^(r) / (n + A)).  Draws use Philox counter
// (q, n, request, TAG_LTR + 256 r) for token q at step n (q = n: the new
// token).
// ---------------------------------------------------------------------------
template <int G>
__device__ void ltr_particle(const DevModel &M, const DevHeldout &H, int64_t d, int32_t r, const float *Rf,
                             uint16_t *mt, TokenZ *tok)
{
    // the count table (K u16, rounded to 16 bytes), then the topic list with
    // room for its windows (launch_heldout sizes the same layout)
    const int32_t Kp = (M.K + 7) & ~7;
    DocState<uint16_t, true> S;
    S.mt = mt;
    S.lst = mt + Kp;
    S.L = 0;
    const int lane = __lane_id();
    const int g = lane & (G - 1);
    const int64_t s = H.doc_off[d];
    const int32_t len = (int32_t)(H.doc_off[d + 1] - s);
    const int64_t base = s * H.R + (int64_t)r * len;
    int32_t *kw = H.kw + base;
    uint16_t *zz = H.z + base;
    double *Zs = H.Zs + base;
    const uint32_t req = H.req[d];
    const uint32_t tag = TAG_LTR + ((uint32_t)r << 8);
    // kept tokens, in order
    int32_t nk = 0;
    for (int32_t p0 = 0; p0 < len; p0 += G) {
        const int32_t p = p0 + g;
        int32_t v = -1;
        bool keep = false;
        if (p < len) {
            v = H.words[s + p];
            keep = v >= 0 && v < M.V && M.colptr[v + 1] > M.colptr[v];
        }
        const uint64_t bal = group_ballot<G>(keep);
        if (keep) kw[nk + __builtin_popcountll(bal & ((1ull << g) - 1ull))] = v;
        nk += __builtin_popcountll(bal);
    }
    if (r == 0 && g == 0) H.kept[d] = nk;
    for (int32_t k = g; k < Kp; k += G) mt[k] = 0;
    // the empty list: every window slot holds the padding value
    for (int32_t j = g; j < win_of<G>() * G + win_of<G>(); j += G) S.lst[j] = (uint16_t)LIST_PAD;
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    ZCount st = {0, 0, 0, 0, 0};
    ZCount32 st32 = {0, 0, 0, 0, 0};
    for (int32_t n = 0; n < nk; ++n) {
        // redraw z_0 .. z_{n-1} in order (lane q mod G stages token q), with
        // the z-step's draw (fp32 b-terms where the rounding bound proves the
        // decision, fp64 elsewhere: the fp64 draws' results)
        for (int32_t q0 = 0; q0 < n; q0 += G) {
            const int32_t q = q0 + g;
            const bool valid = q < n;
            int32_t zo = 0;
            if (valid) {
                zo = zz[q];
                const r4 rr = philox((uint32_t)q, (uint32_t)n, req, tag, H.key0, H.key1);
                // (n tokens counted: the redraws may settle the a-part at
                // staging; only the new token's draw needs its Z)
                stage_token_z(M, tok, g, kw[q], zo, rr, n);
            }
            __builtin_amdgcn_wave_barrier();
            int32_t znew = zo;
            const int nb = n - q0 < G ? n - q0 : G;
            for (int jj = 0; jj < nb; ++jj) {
                const TokenZ tk = tok[jj];
                int32_t k = draw_token_f32<G, uint16_t, true, false>(M, tk, S, Rf, g, 1, st32);
                if (k < 0) k = -1 - k;
                if (g == jj) znew = k;
            }
            __builtin_amdgcn_wave_barrier();
            if (valid) zz[q] = (uint16_t)znew;
        }
        // the new token: counted under a topic the particle already holds
        // (topic 0 at the first step), which the draw removes again, so the
        // draw sees the counts of z_<n
        const int32_t k0 = S.L > 0 ? S.lst[0] : 0;
        const int32_t c0 = mt[k0];
        __builtin_amdgcn_wave_barrier();
        if (g == 0) mt[k0] = (uint16_t)(c0 + 1);
        __builtin_amdgcn_wave_barrier();
        if (c0 == 0) list_insert<G, uint16_t>(S, k0, g);
        // (the fp64 draw, which hands back Z; its R_k from global memory:
        // one such draw per step)
        TokenIn *tin = (TokenIn *)tok;
        if (g == 0) {
            const r4 rr = philox((uint32_t)n, (uint32_t)n, req, tag, H.key0, H.key1);
            stage_token(M, tin, 0, kw[n], k0, rr, 0);
        }
        __builtin_amdgcn_wave_barrier();
        const TokenIn tk = tin[0];
        double Z = 0.0;
        int32_t k = draw_token<G, uint16_t>(M, tk, S, M.Rd, g, 1, st, Z);
        if (k < 0) k = -1 - k;
        __builtin_amdgcn_wave_barrier();
        if (g == (n & (G - 1))) zz[n] = (uint16_t)k;
        if (g == 0) Zs[n] = Z;
    }
}

template <int G>
__global__ void __launch_bounds__(256) ltr_kernel(DevModel M, DevHeldout H, int32_t per_group)
{
    extern __shared__ __align__(16) uint16_t h_lds[];
    float *R = (float *)h_lds;
    for (int32_t k = threadIdx.x; k < M.K; k += blockDim.x) R[k] = (float)M.Rd[k];
    __syncthreads();
    uint16_t *blk = h_lds + (M.K * 4 + 15) / 16 * 8;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    constexpr int NG = 64 / G;
    const int grp = lane / G;
    const int64_t gid = ((int64_t)blockIdx.x * 4 + wave) * NG + grp;
    uint16_t *mt = blk + (wave * NG + grp) * per_group;
    TokenZ *tok = (TokenZ *)(blk + 4 * NG * per_group) + wave * 64 + grp * G;
    if (gid >= H.D * H.R) return;
    ltr_particle<G>(M, H, H.order[gid / H.R], (int32_t)(gid % H.R), R, mt, tok);
}

// one wave per document: sum over steps of log((1/R) sum_r Z_n^(r) / (n + A)),
// the particles added in ascending order
__global__ void __launch_bounds__(256) ltr_finish_kernel(DevHeldout H)
{
    const int64_t d = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (d >= H.D) return;
    const int lane = __lane_id();
    const int64_t s = H.doc_off[d];
    const int32_t len = (int32_t)(H.doc_off[d + 1] - s);
    const int32_t nk = H.kept[d];
    double part = 0.0;
    for (int32_t n = lane; n < nk; n += 64) {
        double sum = 0.0;
        for (int32_t r = 0; r < H.R; ++r) sum += H.Zs[s * H.R + (int64_t)r * len + n] / ((double)n + H.A);
        part += log(sum / (double)H.R);
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if (lane == 0) H.ll[d] = part;
}

hipError_t launch_heldout(const DevModel &m, const DevHeldout &h, hipStream_t s)
{
    if (h.D == 0) return hipSuccess;
    // per particle (u16 units): the count table (K entries), then the topic
    // list (K entries, at least W slots a lane and W more for its windows),
    // each rounded to 16 bytes
    const int32_t W = h.group == 16 ? 8 : 4;
    const int32_t lcap = m.K > W * h.group + W ? m.K : W * h.group + W;
    const int per_group = ((m.K + 7) & ~7) + ((lcap + 7) & ~7);
    const int ngw = 64 / h.group;
    const int64_t groups = h.D * h.R;
    const int64_t waves = (groups + ngw - 1) / ngw;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const size_t lds = (size_t)(m.K * 4 + 15) / 16 * 16 + 4 * ngw * per_group * sizeof(uint16_t) +
                       4 * 64 * sizeof(TokenZ);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ltr_kernel<64>, 256, lds);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) return hipErrorInvalidConfiguration;  // the block's LDS exceeds the CU's
    if (h.group == 64) ltr_kernel<64><<<blocks, 256, lds, s>>>(m, h, per_group);
    else if (h.group == 32) ltr_kernel<32><<<blocks, 256, lds, s>>>(m, h, per_group);
    else ltr_kernel<16><<<blocks, 256, lds, s>>>(m, h, per_group);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ltr_finish_kernel<<<(unsigned)((h.D + 3) / 4), 256, 0, s>>>(h);
    return hipGetLastError();
}

}  // namespace pulda
