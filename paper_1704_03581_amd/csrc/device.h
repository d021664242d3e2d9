// Device helpers for the Polya-urn LDA kernels (gfx950, wave64).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
// from its published definition.  Every draw is addressed by a counter that
// names what is drawn (token index and sweep, or cell and sweep), so results
// never depend on the schedule that computes them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pulda {

enum : uint32_t {
    TAG_INIT = 0,        // initial topic of token i: ctr (i_lo, i_hi, 0, TAG_INIT)
    TAG_PHI_CELL = 1,    // Pois(beta + n_kv) of a counted cell: ctr (v, k, t, TAG_PHI_CELL)
    TAG_PHI_PRIOR = 2,   // j-th geometric jump over column v: ctr (v, j, t, TAG_PHI_PRIOR)
    TAG_Z = 3,           // token draw: ctr (i_lo, i_hi, t, TAG_Z)
    TAG_FOLDIN_INIT = 4, // fold-in initial topic: ctr (p, request, 0, TAG_FOLDIN_INIT)
    TAG_FOLDIN_Z = 5,    // fold-in token draw: ctr (p, request, sweep, TAG_FOLDIN_Z)
    TAG_PHI_GAMMA = 6,   // attempt j of the G(beta + n_kv, 1) draw of cell (k, v) (Algorithm 1's
                         // Phi-step): ctr (v, k, t, TAG_PHI_GAMMA + 256 j)
    TAG_LTR = 7,         // held-out estimate, particle r's draw of kept token q at step n:
                         // ctr (q, n, request, TAG_LTR + 256 r)
};

struct r4 {
    uint32_t x, y, z, w;
};

// Ten rounds of the Philox 4x32 S-box; the key advances by the two Weyl
// constants before every round after the first.
__device__ __forceinline__ r4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t a = 0xD2511F53u * c0, ah = __umulhi(0xD2511F53u, c0);
        const uint32_t b = 0xCD9E8D57u * c2, bh = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = bh ^ c1 ^ k0;
        const uint32_t n2 = ah ^ c3 ^ k1;
        c0 = n0;
        c1 = b;
        c2 = n2;
        c3 = a;
    }
    return {c0, c1, c2, c3};
}

// floor(r * n / 2^32): an integer uniform on [0, n) from one 32-bit word
__device__ __forceinline__ uint32_t scale32(uint32_t r, uint32_t n) { return __umulhi(r, n); }
// 24-bit uniform on [0, 1)
__device__ __forceinline__ double unit24(uint32_t r) { return (double)(r >> 8) * 0x1p-24; }
// 53-bit uniform on [0, 1) from two words
__device__ __forceinline__ double unit53(uint32_t ra, uint32_t rb)
{
    return ((double)(ra >> 5) * 67108864.0 + (double)(rb >> 6)) * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Cross-lane helpers for groups of G lanes (G = 8, 16, 32 or 64) inside a wave.
// Scans use DPP row shifts within 16-lane rows and row broadcasts across
// rows (GFX9 DPP), so a group's scan never reads another group's lanes.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, 0xF, true);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x)
{
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xF, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// inclusive prefix sum over the lanes of a group (ascending lane order);
// a group of 8 is half a row, so its shifted-in values are dropped below
// the shift distance
template <int G>
__device__ __forceinline__ double group_scan_incl(double x)
{
    if constexpr (G == 8) {
        const int gi = __lane_id() & 7;
        double y = dpp_f64<0x111, 0xF>(x);
        x += gi >= 1 ? y : 0.0;
        y = dpp_f64<0x112, 0xF>(x);
        x += gi >= 2 ? y : 0.0;
        y = dpp_f64<0x114, 0xF>(x);
        x += gi >= 4 ? y : 0.0;
        return x;
    }
    x += dpp_f64<0x111, 0xF>(x);  // row_shr:1
    x += dpp_f64<0x112, 0xF>(x);  // row_shr:2
    x += dpp_f64<0x114, 0xF>(x);  // row_shr:4
    x += dpp_f64<0x118, 0xF>(x);  // row_shr:8
    if constexpr (G >= 32) x += dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1, 3
    if constexpr (G >= 64) x += dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2, 3
    return x;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}

// the same scan in fp32 (one DPP add per level)
template <int G>
__device__ __forceinline__ float group_scan_incl_f32(float x)
{
    if constexpr (G == 8) {
        const int gi = __lane_id() & 7;
        float y = dpp_f32<0x111, 0xF>(x);
        x += gi >= 1 ? y : 0.0f;
        y = dpp_f32<0x112, 0xF>(x);
        x += gi >= 2 ? y : 0.0f;
        y = dpp_f32<0x114, 0xF>(x);
        x += gi >= 4 ? y : 0.0f;
        return x;
    }
    x += dpp_f32<0x111, 0xF>(x);
    x += dpp_f32<0x112, 0xF>(x);
    x += dpp_f32<0x114, 0xF>(x);
    x += dpp_f32<0x118, 0xF>(x);
    if constexpr (G >= 32) x += dpp_f32<0x142, 0xA>(x);
    if constexpr (G >= 64) x += dpp_f32<0x143, 0xC>(x);
    return x;
}

template <int G>
__device__ __forceinline__ int group_scan_incl_i32(int x)
{
    if constexpr (G == 8) {
        const int gi = __lane_id() & 7;
        int y = dpp_i32<0x111, 0xF>(x);
        x += gi >= 1 ? y : 0;
        y = dpp_i32<0x112, 0xF>(x);
        x += gi >= 2 ? y : 0;
        y = dpp_i32<0x114, 0xF>(x);
        x += gi >= 4 ? y : 0;
        return x;
    }
    x += dpp_i32<0x111, 0xF>(x);
    x += dpp_i32<0x112, 0xF>(x);
    x += dpp_i32<0x114, 0xF>(x);
    x += dpp_i32<0x118, 0xF>(x);
    if constexpr (G >= 32) x += dpp_i32<0x142, 0xA>(x);
    if constexpr (G >= 64) x += dpp_i32<0x143, 0xC>(x);
    return x;
}

// value of lane `src` (group-relative) to every lane of the group
template <int G>
__device__ __forceinline__ int group_bcast(int x, int src)
{
    if constexpr (G == 64) {
        return __builtin_amdgcn_readlane(x, src);
    } else {
        return __shfl(x, src, G);
    }
}

template <int G>
__device__ __forceinline__ float group_bcast_f32(float x, int src)
{
    return __int_as_float(group_bcast<G>(__float_as_int(x), src));
}

template <int G>
__device__ __forceinline__ double group_bcast_f64(double x, int src)
{
    int lo = group_bcast<G>(__double2loint(x), src);
    int hi = group_bcast<G>(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}

// bitmask of the group's lanes for which pred holds (bit g = group lane g)
template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool pred)
{
    const uint64_t all = __builtin_amdgcn_ballot_w64(pred);
    if constexpr (G == 64) {
        return all;
    } else if constexpr (G == 32) {
        return __lane_id() < 32 ? (uint32_t)all : (uint32_t)(all >> 32);
    } else {
        const int base = (int)(__lane_id() & ~(G - 1));
        return (all >> base) & ((1ull << G) - 1ull);
    }
}

}  // namespace pulda
