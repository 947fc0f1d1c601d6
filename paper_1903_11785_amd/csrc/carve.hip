// Silhouette packing and volumetric visual-hull carving (Sec. II-B-1 over the
// whole volume, Sec. II-B-3 inside ROIs) for gfx950.
//
// A workgroup of 256 threads carves a tile of TX x TY x TZ lattice samples
// (TX * TY = 256).  The tile keeps, in LDS, the list of its samples that are
// still inside every camera tested so far.  Each pass tests the listed samples
// against the next kCamGroup cameras (independent loads, one memory round trip
// per pass) and appends the survivors to the other list, so every lane of a
// pass works on a live sample: samples outside the lattice never enter the
// list and rejected ones leave it at once.  The tile is done when a pass
// leaves no survivor or the cameras run out; the survivors are the occupied
// samples.  The occupancy is the AND over all cameras, so neither the passes
// nor the order in which samples are listed change a result.  Each test
// evaluates the full fused projection chain of the sample, bit-equal to the
// definition.
#include "fvv_internal.h"

#include <type_traits>

namespace fvv {

constexpr int kCamGroup = 2;

// ------------------------------------------------------------------ packing
// Non-zero flags of the four bytes of x as bits 0..3.  Adding 0x7f to a
// byte's low seven bits sets its high bit iff they are not all zero (no carry
// leaves the byte); ORed with the byte's own high bit, that bit says the byte
// is non-zero.  Shifted to bits 0, 8, 16, 24, the flags are gathered into bits
// 21..24 by one multiply by 1 + 2^7 + 2^14 + 2^21 (no two partial products
// share a bit there).
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
    const uint32_t f = ((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) >> 7) & 0x01010101u;
    return ((f * 0x00204081u) >> 21) & 0xfu;
}

// Unsigned 32-bit division by a fixed divisor d >= 1 with a host-computed
// multiplier (the round-up method of Granlund and Montgomery, exact for every
// 32-bit dividend): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), t = (n m) >> 32.
struct DivU32 {
    uint32_t m;
    int s1, s2;
};

DivU32 divu32_magic(uint32_t d) {
    int l = 0;
    while (l < 32 && (1ull << l) < d)
        ++l;
    const uint64_t m = (((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1;
    return DivU32{(uint32_t)m, l < 1 ? l : 1, l > 1 ? l - 1 : 0};
}

__device__ __forceinline__ uint32_t divu32(uint32_t n, const DivU32& d) {
    const uint32_t t = __umulhi(n, d.m);
    return (t + ((n - t) >> d.s1)) >> d.s2;
}

// One lane per 32-pixel word.  Fast path: rows of a multiple of 32 pixels
// whose 32 bytes per word are read with two 16-byte loads.  k32: every word
// index fits 32 bits (row = index / wpr by multiply and shifts).
template <bool k32>
__global__ __launch_bounds__(kBlock) void pack_kernel(const uint8_t* __restrict__ masks,
                                                      uint32_t* __restrict__ sils, int n, int W,
                                                      int H, int wpr, DivU32 by_wpr) {
    const int64_t total = (int64_t)n * H * wpr;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t row;
        if (k32)
            row = divu32((uint32_t)idx, by_wpr);
        else
            row = idx / wpr;
        const int word = (int)(idx - row * wpr);
        const uint8_t* src = masks + row * W + (int64_t)word * 32;
        uint32_t bits = 0;
        if ((W & 31) == 0) {
            const uint4* v = reinterpret_cast<const uint4*>(src);
            uint4 q[2] = {v[0], v[1]};
            const uint32_t* d = reinterpret_cast<const uint32_t*>(q);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                bits |= nonzero_bytes(d[k]) << (4 * k);
        } else {
            int nb = min(32, W - word * 32);
            for (int b = 0; b < nb; ++b)
                bits |= (uint32_t)(src[b] != 0) << b;
        }
        sils[idx] = bits;
    }
}

hipError_t launch_pack(int n, int W, int H, const uint8_t* masks, uint32_t* sils, hipStream_t s) {
    int wpr = (W + 31) / 32;
    int64_t total = (int64_t)n * H * wpr;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    if (blocks < 1)
        blocks = 1;
    const DivU32 dw = divu32_magic((uint32_t)wpr);
    // 32-bit indices while every index the grid-stride loop forms stays below 2^32
    if (total + (int64_t)blocks * kBlock <= ((int64_t)1 << 32))
        hipLaunchKernelGGL(pack_kernel<true>, dim3((unsigned)blocks), dim3(kBlock), 0, s, masks,
                           sils, n, W, H, wpr, dw);
    else
        hipLaunchKernelGGL(pack_kernel<false>, dim3((unsigned)blocks), dim3(kBlock), 0, s, masks,
                           sils, n, W, H, wpr, dw);
    return hipGetLastError();
}

// ------------------------------------------------------------------ tiled silhouettes
// The silhouettes in 8 x 8-pixel blocks, one uint64 per block: pixel (x, y) at
// bit 8 (y & 7) + (x & 7) of block (x / 8, y / 8); blocks row-major per camera,
// block (bx, by) of camera c at c * tpc + by * tpr + bx with tpr = ceil(W / 8)
// and tpc = tpr * ceil(H / 8).  Pixels past the image are 0.  A pixel rectangle
// of up to 9 x 9 pixels lies in at most 2 x 2 blocks.
//
// Both kernels below run one thread per block; with kAny they also OR each
// non-empty block's bit into its SilAny word (all-zero before).

// From the packed rows (whose padding bits are 0).
template <bool kAny>
__global__ __launch_bounds__(kBlock) void tile_sils_kernel(const uint32_t* __restrict__ sils,
                                                           int n, int H, int wpr, int tpr,
                                                           int tph, int bw,
                                                           uint64_t* __restrict__ tiles,
                                                           uint64_t* __restrict__ any) {
    const int64_t total = (int64_t)n * tph * tpr;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t cb = idx / tpr;                  // camera * tph + block row
        const int bx = (int)(idx - cb * tpr);
        const int c = (int)(cb / tph), by = (int)(cb - (int64_t)c * tph);
        const uint32_t* col = sils + (int64_t)c * H * wpr + (bx >> 2);
        const int sh = 8 * (bx & 3);
        uint64_t v = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int y = 8 * by + r;
            if (y < H)
                v |= (uint64_t)((col[(int64_t)y * wpr] >> sh) & 0xffu) << (8 * r);
        }
        tiles[idx] = v;
        if (kAny && v != 0)
            atomicOr((unsigned long long*)&any[cb * bw + (bx >> 6)], 1ull << (bx & 63));
    }
}


// Both forms at once, straight from the masks, for images whose width is a
// multiple of 8: each block's thread reads its 8 rows of 8 bytes (a wave
// covers 512 contiguous bytes of each row), stores the block's word and the
// block's byte of each of its 8 packed rows (the row's last block also clears
// the padding bytes of the row's last word).  k32: every block index fits 32
// bits (split by multiply and shifts).
template <bool k32, bool kAny>
__global__ __launch_bounds__(kBlock) void pack_tiled_kernel(const uint8_t* __restrict__ masks,
                                                            int n, int W, int H, int wpr,
                                                            int tpr, int tph, int bw,
                                                            DivU32 by_tpr, DivU32 by_tph,
                                                            uint32_t* __restrict__ sils,
                                                            uint64_t* __restrict__ tiles,
                                                            uint64_t* __restrict__ any) {
    const int64_t total = (int64_t)n * tph * tpr;
    uint8_t* const rows = reinterpret_cast<uint8_t*>(sils);
    const int row_bytes = 4 * wpr;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t cb, c;
        if (k32) {
            cb = divu32((uint32_t)idx, by_tpr);
            c = divu32((uint32_t)cb, by_tph);
        } else {
            cb = idx / tpr;
            c = cb / tph;
        }
        const int bx = (int)(idx - cb * tpr);
        const int by = (int)(cb - c * tph);
        const int y0 = 8 * by;
        const int nr = min(8, H - y0);
        const uint8_t* src = masks + ((int64_t)c * H + y0) * W + 8 * bx;
        uint8_t* dst = rows + ((int64_t)c * H + y0) * row_bytes + bx;
        uint64_t v = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r < nr) {
                const uint2 q = *reinterpret_cast<const uint2*>(src + (int64_t)r * W);
                const uint32_t b = nonzero_bytes(q.x) | (nonzero_bytes(q.y) << 4);
                v |= (uint64_t)b << (8 * r);
                dst[(int64_t)r * row_bytes] = (uint8_t)b;
                if (bx == tpr - 1)
                    for (int k = tpr; k < row_bytes; ++k)
                        dst[(int64_t)r * row_bytes + (k - bx)] = 0;
            }
        }
        tiles[idx] = v;
        if (kAny && v != 0)
            atomicOr((unsigned long long*)&any[cb * bw + (bx >> 6)], 1ull << (bx & 63));
    }
}

// The same for images whose width is a multiple of 16 (masks 16-byte
// aligned): one thread per two horizontally adjacent blocks, 16-byte loads of
// its 8 rows, the two blocks' words in one 16-byte store and two bytes of
// each packed row in one 2-byte store.
template <bool k32, bool kAny>
__global__ __launch_bounds__(kBlock) void pack_tiled16_kernel(const uint8_t* __restrict__ masks,
                                                              int n, int W, int H, int wpr,
                                                              int tpr, int tph, int bw,
                                                              DivU32 by_tp2, DivU32 by_tph,
                                                              uint32_t* __restrict__ sils,
                                                              uint64_t* __restrict__ tiles,
                                                              uint64_t* __restrict__ any) {
    const int tp2 = tpr / 2;
    const int64_t total = (int64_t)n * tph * tp2;
    uint8_t* const rows = reinterpret_cast<uint8_t*>(sils);
    const int row_bytes = 4 * wpr;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        int64_t cb, c;
        if (k32) {
            cb = divu32((uint32_t)idx, by_tp2);
            c = divu32((uint32_t)cb, by_tph);
        } else {
            cb = idx / tp2;
            c = cb / tph;
        }
        const int bx = 2 * (int)(idx - cb * tp2);
        const int by = (int)(cb - c * tph);
        const int y0 = 8 * by;
        const int nr = min(8, H - y0);
        const uint8_t* src = masks + ((int64_t)c * H + y0) * W + 8 * bx;
        uint8_t* dst = rows + ((int64_t)c * H + y0) * row_bytes + bx;
        uint64_t v0 = 0, v1 = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r < nr) {
                const uint4 q = *reinterpret_cast<const uint4*>(src + (int64_t)r * W);
                const uint32_t b0 = nonzero_bytes(q.x) | (nonzero_bytes(q.y) << 4);
                const uint32_t b1 = nonzero_bytes(q.z) | (nonzero_bytes(q.w) << 4);
                v0 |= (uint64_t)b0 << (8 * r);
                v1 |= (uint64_t)b1 << (8 * r);
                *reinterpret_cast<uint16_t*>(dst + (int64_t)r * row_bytes) =
                    (uint16_t)(b0 | (b1 << 8));
                if (bx == tpr - 2)
                    for (int k = tpr; k < row_bytes; ++k)
                        dst[(int64_t)r * row_bytes + (k - bx)] = 0;
            }
        }
        *reinterpret_cast<ulonglong2*>(tiles + cb * tpr + bx) = make_ulonglong2(v0, v1);
        if (kAny && (v0 | v1) != 0)
            atomicOr((unsigned long long*)&any[cb * bw + (bx >> 6)],
                     (unsigned long long)((v0 ? 1ull : 0ull) | (v1 ? 2ull : 0ull)) << (bx & 63));
    }
}

hipError_t launch_pack_tiled(int n, int W, int H, const uint8_t* masks, uint32_t* sils,
                             uint64_t* tiles, uint64_t* any, hipStream_t s) {
    if (W % 8 != 0 || reinterpret_cast<uintptr_t>(masks) % 8 != 0) {
        hipError_t e = launch_pack(n, W, H, masks, sils, s);
        return e == hipSuccess ? launch_tile_sils(n, W, H, sils, tiles, any, s) : e;
    }
    const int wpr = (W + 31) / 32, tpr = W / 8, tph = (H + 7) / 8, bw = sil_any_bw(W);
    if (W % 16 == 0 && reinterpret_cast<uintptr_t>(masks) % 16 == 0) {
        const int64_t total = (int64_t)n * tph * (tpr / 2);
        int64_t blocks = (total + kBlock - 1) / kBlock;
        blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
        const DivU32 dx = divu32_magic((uint32_t)(tpr / 2)), dy = divu32_magic((uint32_t)tph);
        const bool k32 = total + (int64_t)blocks * kBlock <= ((int64_t)1 << 32);
        auto kernel = k32 ? (any ? pack_tiled16_kernel<true, true> : pack_tiled16_kernel<true, false>)
                          : (any ? pack_tiled16_kernel<false, true>
                                 : pack_tiled16_kernel<false, false>);
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, masks, n, W, H,
                           wpr, tpr, tph, bw, dx, dy, sils, tiles, any);
        return hipGetLastError();
    }
    const int64_t total = (int64_t)n * tph * tpr;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
    const DivU32 dx = divu32_magic((uint32_t)tpr), dy = divu32_magic((uint32_t)tph);
    const bool k32 = total + (int64_t)blocks * kBlock <= ((int64_t)1 << 32);
    auto kernel = k32 ? (any ? pack_tiled_kernel<true, true> : pack_tiled_kernel<true, false>)
                      : (any ? pack_tiled_kernel<false, true> : pack_tiled_kernel<false, false>);
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, masks, n, W, H, wpr,
                       tpr, tph, bw, dx, dy, sils, tiles, any);
    return hipGetLastError();
}


hipError_t launch_tile_sils(int n, int W, int H, const uint32_t* sils, uint64_t* tiles,
                            uint64_t* any, hipStream_t s) {
    const int wpr = (W + 31) / 32, tpr = (W + 7) / 8, tph = (H + 7) / 8, bw = sil_any_bw(W);
    const int64_t total = (int64_t)n * tph * tpr;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
    hipLaunchKernelGGL(any ? tile_sils_kernel<true> : tile_sils_kernel<false>,
                       dim3((unsigned)blocks), dim3(kBlock), 0, s, sils, n, H, wpr, tpr, tph, bw,
                       tiles, any);
    return hipGetLastError();
}

// ------------------------------------------------------------------ carving tile
constexpr int log2_of(int v) { return v <= 1 ? 0 : 1 + log2_of(v / 2); }

// Append val to an LDS list for the lanes where pred holds (one LDS atomic
// per wave).
__device__ __forceinline__ void lds_append(bool pred, uint16_t val, uint16_t* list,
                                           uint32_t* count) {
    const uint64_t m = __ballot(pred);
    if (m == 0)
        return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader)
        base = atomicAdd(count, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if (pred)
        list[base + lane_rank(m)] = val;
}

// Where the carve also writes its occupancy as bits: nowhere, ORed into the
// labelling's row bitmap (RowBits, all-zero before), or stored into a fine
// bitmap (rows padded to words, every word of the lattice written).
constexpr int kBitsNone = 0, kBitsLabel = 1, kBitsFine = 2;

// Carve tile `tile` of lattice g.  getP(c) returns camera c's 12 floats (a
// wave-uniform address); sil_of(c) its silhouette rows.  The TX lanes of one
// tile row cover TX consecutive x inside one bitmap word (TX divides 64), so a
// tile row's bits cost one atomic (kBitsLabel, none where the row is empty)
// or one store (kBitsFine).
template <int TX, int TZ, int kBits, typename GetP, typename GetSil>
__device__ __forceinline__ void carve_tile(GetP getP, GetSil sil_of, int ncam, int W, int H,
                                           int wpr, const fvv_grid& g, uint64_t tile,
                                           uint8_t* __restrict__ out, const RowBits& rb) {
    constexpr int TY = kBlock / TX;
    constexpr int TV = TX * TY * TZ;
    constexpr int LX = log2_of(TX), LY = log2_of(TY);
    __shared__ uint16_t s_list[2][TV];
    __shared__ uint32_t s_cnt[3];
    __shared__ uint32_t s_alive[TV / 32];

    const int ntx = (g.dims[0] + TX - 1) / TX;
    const int nty = (g.dims[1] + TY - 1) / TY;
    const int bx = (int)(tile % (uint64_t)ntx);
    const uint64_t r = tile / (uint64_t)ntx;
    const int by = (int)(r % (uint64_t)nty);
    const int bz = (int)(r / (uint64_t)nty);
    const int i0 = bx * TX, j0 = by * TY, k0 = bz * TZ;

    __syncthreads();   // the previous tile of this workgroup is done with the LDS
    if (threadIdx.x < 3)
        s_cnt[threadIdx.x] = 0;
    for (int w = threadIdx.x; w < TV / 32; w += kBlock)
        s_alive[w] = 0;
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < TZ; ++rr) {
        const int s = rr * kBlock + (int)threadIdx.x;
        const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
        const bool valid = i0 + lx < g.dims[0] && j0 + ly < g.dims[1] && k0 + lz < g.dims[2];
        lds_append(valid, (uint16_t)s, s_list[0], &s_cnt[0]);
    }
    __syncthreads();

    int cur = 0;
    for (int c0 = 0; c0 < ncam; c0 += kCamGroup) {
        const uint32_t n = s_cnt[cur % 3];
        if (n == 0)
            break;
        if (threadIdx.x == 0)
            s_cnt[(cur + 2) % 3] = 0;   // last read a pass ago, next appended to a pass on
        const float* P[kCamGroup];
        const uint32_t* sil[kCamGroup];
#pragma unroll
        for (int q = 0; q < kCamGroup; ++q) {
            const int c = c0 + q < ncam ? c0 + q : c0;   // wave-uniform
            P[q] = getP(c);
            sil[q] = sil_of(c);
        }
        const uint16_t* src = s_list[cur & 1];
        uint16_t* dst = s_list[(cur + 1) & 1];
        uint32_t* dcnt = &s_cnt[(cur + 1) % 3];
        // each wave takes 64 consecutive entries per round and stops as soon
        // as its next slice starts past the end of the list
        const uint32_t wave0 = (threadIdx.x / kWave) * kWave;
        for (uint32_t base = wave0; base < n; base += kBlock) {
            const uint32_t idx = base + lane_id();
            const bool act = idx < n;
            const int s = act ? src[idx] : 0;
            const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
            const float X = lattice_coord(g.lo[0] + i0 + lx, g.h, g.origin[0]);
            const float Y = lattice_coord(g.lo[1] + j0 + ly, g.h, g.origin[1]);
            const float Z = lattice_coord(g.lo[2] + k0 + lz, g.h, g.origin[2]);
            // all tests of the group are issued unconditionally (a camera past
            // the last one repeats camera c0 and cannot change the result), so
            // their silhouette loads are in flight together
            const bool in = group_inside<kCamGroup>(P, X, Y, Z, sil, W, H, wpr);
            lds_append(act && in, (uint16_t)s, dst, dcnt);
        }
        __syncthreads();
        ++cur;
    }

    const uint32_t n_in = s_cnt[cur % 3];
    const uint16_t* surv = s_list[cur & 1];
    for (uint32_t base = 0; base < n_in; base += kBlock) {
        const uint32_t idx = base + threadIdx.x;
        const bool act = idx < n_in;
        const int s = act ? surv[idx] : 0;
        if (act)
            atomicOr(&s_alive[s >> 5], 1u << (s & 31));
    }
    __syncthreads();
    const uint64_t plane = (uint64_t)g.dims[0] * (uint64_t)g.dims[1];
#pragma unroll
    for (int rr = 0; rr < TZ; ++rr) {
        const int s = rr * kBlock + (int)threadIdx.x;
        const int lx = s & (TX - 1), ly = (s >> LX) & (TY - 1), lz = s >> (LX + LY);
        const int i = i0 + lx, j = j0 + ly, k = k0 + lz;
        const bool valid = i < g.dims[0] && j < g.dims[1] && k < g.dims[2];
        const uint32_t bit = (s_alive[s >> 5] >> (s & 31)) & 1u;
        if (valid)
            out[(uint64_t)k * plane + (uint64_t)j * g.dims[0] + i] = (uint8_t)bit;
        if (kBits != kBitsNone) {
            // lanes [TX*q, TX*q + TX) of the wave hold one tile row (lx = 0..TX-1)
            const uint64_t m = __ballot(valid && bit != 0u);
            const int q = lane_id() / TX;
            const uint64_t bits = TX == 64 ? m : (m >> (q * TX)) & ((1ull << (TX & 63)) - 1);
            const int64_t row = (int64_t)j + (int64_t)g.dims[1] * k;
            uint64_t* word = rb.words + row * rb.wr + (i0 >> 6);
            if (kBits == kBitsLabel && lx == 0 && bits != 0) {
                atomicOr((unsigned long long*)word, (unsigned long long)(bits << (i0 & 63)));
                atomicOr((unsigned long long*)&rb.rowmask[row >> 6], 1ull << (row & 63));
            }
            if (kBits == kBitsFine && lx == 0 && j < g.dims[1] && k < g.dims[2]) {
                if (TX == 64)
                    *word = bits;
                else if (TX == 32)
                    reinterpret_cast<uint32_t*>(word)[(i0 >> 5) & 1] = (uint32_t)bits;
                else
                    reinterpret_cast<uint16_t*>(word)[(i0 >> 4) & 3] = (uint16_t)bits;
            }
        }
    }
}

// ------------------------------------------------------------------ batched, persistent
// A job of a batched carve that the kernels can carve: 1..FVV_MAX_CAMS cameras
// of a valid image size, a non-empty lattice and non-negative offsets.
__device__ __forceinline__ bool job_ok(const fvv_job& j) {
    return j.n_cams >= 1 && j.n_cams <= FVV_MAX_CAMS && j.width >= 1 && j.height >= 1 &&
           j.width <= (1 << 16) && j.height <= (1 << 16) && j.grid.dims[0] >= 1 &&
           j.grid.dims[1] >= 1 && j.grid.dims[2] >= 1 && j.cam_base >= 0 && j.sil_base >= 0 &&
           j.out_offset >= 0;
}

// Prefix sums of tile and tile-row counts over a host-given job table; resets
// the work counter.  counter[0] = next work item, [1] = tiles per item,
// [2] = jobs.  A job out of range gets no tiles and raises the job flag.
template <int TX, int TZ>
__global__ __launch_bounds__(kBlock) void batched_prepare_kernel(const fvv_job* __restrict__ jobs,
                                                                 uint32_t n_jobs,
                                                                 JobPrefix* __restrict__ pre,
                                                                 uint32_t* __restrict__ counter,
                                                                 uint32_t* __restrict__ status,
                                                                 uint32_t blocks) {
    __shared__ uint64_t scratch[kBlock / kWave];
    __shared__ uint64_t carry, carry_rows;
    if (threadIdx.x == 0) {
        carry = 0;
        carry_rows = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < n_jobs; base += kBlock) {
        uint32_t j = base + threadIdx.x;
        uint64_t t = 0, rows = 0;
        if (j < n_jobs) {
            if (job_ok(jobs[j])) {
                t = tiles_of_grid(jobs[j].grid, TX, TZ);
                rows = t / (uint64_t)((jobs[j].grid.dims[0] + TX - 1) / TX);
            } else {
                atomicOr(status, kFlagJob);
            }
        }
        uint64_t tot, tot_rows;
        const uint64_t ex = block_exclusive_sum64<kBlock>(t, scratch, &tot);
        const uint64_t ex_rows = block_exclusive_sum64<kBlock>(rows, scratch, &tot_rows);
        const uint64_t c0 = carry, r0 = carry_rows;
        if (j < n_jobs) {
            pre[j].tile_off = c0 + ex;
            pre[j].row_off = r0 + ex_rows;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry = c0 + tot;
            carry_rows = r0 + tot_rows;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t total = carry;
        pre[n_jobs].tile_off = total;
        pre[n_jobs].row_off = carry_rows;
        counter[0] = 0;
        counter[1] = grab_size(total, blocks);
        counter[2] = n_jobs;
    }
}

// Rounding pad of every (job, camera) pair over the job's lattice box, for the
// camera culling of the batched carve: job_pad[j * FVV_MAX_CAMS + c].
__global__ __launch_bounds__(kBlock) void job_pad_kernel(const fvv_job* __restrict__ jobs,
                                                         uint32_t n_jobs,
                                                         const fvv_camera* __restrict__ cams,
                                                         float* __restrict__ job_pad) {
    const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= (uint64_t)n_jobs * FVV_MAX_CAMS)
        return;
    const fvv_job& j = jobs[p / FVV_MAX_CAMS];
    const int c = (int)(p % FVV_MAX_CAMS);
    if (!job_ok(j) || c >= j.n_cams)
        return;
    double lo[3], hi[3];
    grid_box(j.grid, lo, hi);
    job_pad[p] = rounding_pad(cams[j.cam_base + c].P, j.width, j.height, lo, hi);
}

template <int TX, int TZ, bool kFineBits>
__global__ __launch_bounds__(kBlock) void carve_persistent_kernel(
    const fvv_job* __restrict__ jobs, const JobPrefix* __restrict__ pre,
    uint32_t* __restrict__ counter, const fvv_camera* __restrict__ cams,
    const uint32_t* __restrict__ sils, uint8_t* __restrict__ out, uint64_t* __restrict__ finebits) {
    __shared__ uint32_t s_item;
    const uint32_t nj = counter[2];
    const uint64_t per = counter[1];
    const uint64_t total = pre[nj].tile_off;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = atomicAdd(&counter[0], 1u);
        __syncthreads();
        const uint64_t t0 = (uint64_t)s_item * per;
        __syncthreads();
        if (t0 >= total)
            break;
        const uint64_t t1 = t0 + per < total ? t0 + per : total;
        for (uint64_t t = t0; t < t1; ++t) {
            const int jb = upper_job([&](int m) { return pre[m].tile_off; }, (int)nj, t);
            const fvv_job job = jobs[jb];
            const int wpr = (job.width + 31) / 32;
            const int64_t cam_words = (int64_t)job.height * wpr;
            const fvv_camera* jc = cams + job.cam_base;
            const uint32_t* js = sils + job.sil_base;
            RowBits fb{};
            if (kFineBits) {
                fb.words = finebits + pre[jb].bit_off;
                fb.wr = (job.grid.dims[0] + 63) / 64;
            }
            carve_tile<TX, TZ, kFineBits ? kBitsFine : kBitsNone>(
                [&](int c) { return &jc[c].P[0]; }, [&](int c) { return js + c * cam_words; },
                job.n_cams, job.width, job.height, wpr, job.grid, t - pre[jb].tile_off,
                out + job.out_offset, fb);
        }
    }
}

// ------------------------------------------------------------------ frame fine carve, culled
// The fine carve of a frame classifies cameras per box of lattice samples
// before testing samples.  The projections of a box's samples lie in the
// convex hull of its eight corner projections (w > 0 over the whole lattice
// box wherever the rounding pad is finite), and the pad bounds how far a
// sample's floored quotient and the corners' rcp quotients can be from the
// real projections; so every sample's pixel lies in the corners' pixel
// rectangle widened by the pad.  If that rectangle holds no foreground pixel
// of the image, the camera rejects every sample of the box; if it lies inside
// the image and is all foreground, it accepts every sample.  Otherwise the
// camera is mixed for the box and its samples are tested one by one.  A tile
// (TX x TY x 4) is classified as 16 sub-blocks of 4 x 4 x 4 samples, one
// (sub-block, camera) pair per thread; one wave then carves one sub-block,
// lane = sample, testing only the sub-block's mixed cameras.  Results are
// identical to testing every camera: the skipped tests are decided by the
// rectangles.
constexpr int kCullMixed = 0, kCullAccept = 1, kCullReject = 2;

// Pixel rectangle from the corner quotient bounds [x0, x1] x [y0, y1] of a
// box: widened by the rounding pad, clamped a little outside the image (which
// keeps the conversions exact) and then to the image.  Returns kCullMixed when
// no pad bound holds, kCullReject when the rectangle misses the image, else -1
// with the clamped rectangle [cx0, cx1] x [cy0, cy1] and whether the unclamped
// one lies inside the image.
__device__ __forceinline__ int rect_of_bounds(float x0, float x1, float y0, float y1, float pad,
                                              int Wi, int Hi, int& cx0, int& cx1, int& cy0,
                                              int& cy1, bool& inside) {
    if (!(pad < 1.0f))
        return kCullMixed;
    const float W = (float)Wi, H = (float)Hi;
    const int px0 = (int)__builtin_floorf(__builtin_amdgcn_fmed3f(x0 - pad, -2.0f, W + 1.0f));
    const int px1 = (int)__builtin_floorf(__builtin_amdgcn_fmed3f(x1 + pad, -2.0f, W + 1.0f));
    const int py0 = (int)__builtin_floorf(__builtin_amdgcn_fmed3f(y0 - pad, -2.0f, H + 1.0f));
    const int py1 = (int)__builtin_floorf(__builtin_amdgcn_fmed3f(y1 + pad, -2.0f, H + 1.0f));
    inside = px0 >= 0 && py0 >= 0 && px1 < Wi && py1 < Hi;
    cx0 = max(px0, 0);
    cx1 = min(px1, Wi - 1);
    cy0 = max(py0, 0);
    cy1 = min(py1, Hi - 1);
    if (cx0 > cx1 || cy0 > cy1)
        return kCullReject;                    // every sample projects off the image
    return -1;
}

// Quotients of camera P at one corner of the box lo, hi (bit a of `corner`
// picks hi on axis a), with an rcp-based division.
__device__ __forceinline__ void corner_quotients(const float* P, const float* lo, const float* hi,
                                                 int corner, float& qa, float& qb) {
    const float X = (corner & 1) ? hi[0] : lo[0];
    const float Y = (corner & 2) ? hi[1] : lo[1];
    const float Z = (corner & 4) ? hi[2] : lo[2];
    const float a = __builtin_fmaf(P[2], Z, __builtin_fmaf(P[1], Y, __builtin_fmaf(P[0], X, P[3])));
    const float b = __builtin_fmaf(P[6], Z, __builtin_fmaf(P[5], Y, __builtin_fmaf(P[4], X, P[7])));
    const float w =
        __builtin_fmaf(P[10], Z, __builtin_fmaf(P[9], Y, __builtin_fmaf(P[8], X, P[11])));
    const float r = __builtin_amdgcn_rcpf(w);
    qa = a * r;
    qb = b * r;
}

// Pixel rectangle of camera c over the box of samples with world corners lo,
// hi (see rect_of_bounds).
template <class Cams>
__device__ __forceinline__ int box_rect(const Cams& cams, int c, const float* lo, const float* hi,
                                        int& cx0, int& cx1, int& cy0, int& cy1, bool& inside) {
    const float pad = cams.padc(c);
    if (!(pad < 1.0f))
        return kCullMixed;
    const float* P = cams.Pc(c);
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float qa, qb;
        corner_quotients(P, lo, hi, k, qa, qb);
        x0 = fminf(x0, qa);
        x1 = fmaxf(x1, qa);
        y0 = fminf(y0, qb);
        y1 = fmaxf(y1, qb);
    }
    return rect_of_bounds(x0, x1, y0, y1, pad, cams.W, cams.H, cx0, cx1, cy0, cy1, inside);
}

// Lane permutations within aligned groups of 8 lanes (DPP): swap neighbours,
// swap pairs, swap quads.
template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, false));
}

__device__ __forceinline__ float min8(float v) {
    v = fminf(v, dpp_f32<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fminf(v, dpp_f32<0x4E>(v));    // quad_perm [2,3,0,1]
    return fminf(v, dpp_f32<0x141>(v));  // row_half_mirror
}

__device__ __forceinline__ float max8(float v) {
    v = fmaxf(v, dpp_f32<0xB1>(v));
    v = fmaxf(v, dpp_f32<0x4E>(v));
    return fmaxf(v, dpp_f32<0x141>(v));
}

// Foreground test of row y of silhouette `sil` over columns [cx0, cx1], at
// most kWords words from word w0: any / all of the pixels set.
template <int kWords>
__device__ __forceinline__ void row_any_all(const uint32_t* __restrict__ row, int cx0, int cx1,
                                            bool on, bool& any, bool& all) {
    const int w0 = cx0 >> 5, w1 = cx1 >> 5;
#pragma unroll
    for (int q = 0; q < kWords; ++q) {
        const int wq = w0 + q;
        const bool won = on && wq <= w1;
        const uint32_t lo_m = wq == w0 ? ~0u << (cx0 & 31) : ~0u;
        const uint32_t hi_m = wq == w1 ? (~0u >> (31 - (cx1 & 31))) : ~0u;
        const uint32_t m = won ? (lo_m & hi_m) : 0u;
        uint32_t v = 0;
        if (won)
            v = row[wq];
        any |= (v & m) != 0u;
        all &= (v & m) == m;
    }
}

// Classification of camera c for the box of samples with world corners lo,
// hi: rectangles of more than kRows rows or kWords silhouette words count as
// mixed.
template <int kRows, int kWords, class Cams>
__device__ __forceinline__ int classify_box(const Cams& cams, int c,
                                            const uint32_t* __restrict__ sil, const float* lo,
                                            const float* hi) {
    int cx0, cx1, cy0, cy1;
    bool inside;
    const int r0 = box_rect(cams, c, lo, hi, cx0, cx1, cy0, cy1, inside);
    if (r0 >= 0)
        return r0;
    if (cy1 - cy0 >= kRows || (cx1 >> 5) - (cx0 >> 5) >= kWords)
        return kCullMixed;
    bool any = false, all = true;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const bool row_on = r <= cy1 - cy0;
        row_any_all<kWords>(sil + (row_on ? cy0 + r : cy0) * cams.wpr, cx0, cx1, row_on, any,
                            all);
    }
    if (!any)
        return kCullReject;
    return (inside && all) ? kCullAccept : kCullMixed;
}

// Classification of every camera for the box lo, hi by one wave, four cameras
// per pass: the 16 lanes of camera cb + l/16 project one corner each (lanes
// l%8) and reduce the corner bounds over 8 lanes, then test row l%16 of the
// rectangle (rectangles of more than 16 rows or kWords words count as mixed).
// Returns, uniform over the wave, the cameras that reject every sample of the
// box and those that are mixed; the others accept every sample.
template <int kWords, class Cams>
__device__ __forceinline__ void classify_box_wave(const Cams& cams,
                                                  const uint32_t* __restrict__ sils,
                                                  int64_t cam_words, const float* lo,
                                                  const float* hi, uint32_t& reject,
                                                  uint32_t& mixed) {
    const int lane = lane_id(), r = lane & 15, grp = lane >> 4;
    reject = 0;
    mixed = 0;
    for (int cb = 0; cb < cams.n; cb += 4) {
        const int c = cb + grp;
        const bool cam_on = c < cams.n;
        const int cc = cam_on ? c : cb;
        float qa, qb;
        corner_quotients(cams.Pc(cc), lo, hi, lane & 7, qa, qb);
        const float x0 = min8(qa), x1 = max8(qa), y0 = min8(qb), y1 = max8(qb);
        int cx0, cx1, cy0, cy1;
        bool inside = false;
        int st = rect_of_bounds(x0, x1, y0, y1, cams.padc(cc), cams.W, cams.H, cx0, cx1, cy0, cy1,
                                inside);
        if (st < 0 && (cy1 - cy0 >= 16 || (cx1 >> 5) - (cx0 >> 5) >= kWords))
            st = kCullMixed;
        bool any = false, all = true;
        if (cam_on && st < 0) {
            const bool row_on = r <= cy1 - cy0;
            row_any_all<kWords>(sils + cc * cam_words + (row_on ? cy0 + r : cy0) * cams.wpr, cx0,
                                cx1, row_on, any, all);
        }
        const uint32_t gany = (uint32_t)(__ballot(any) >> (16 * grp)) & 0xffffu;
        const uint32_t gall = (uint32_t)(__ballot(all) >> (16 * grp)) & 0xffffu;
        const bool rej = cam_on && (st == kCullReject || (st < 0 && gany == 0));
        const bool acc = cam_on && st < 0 && gany != 0 && inside && gall == 0xffffu;
        const uint64_t rb = __ballot(r == 0 && rej), mb = __ballot(r == 0 && cam_on && !rej && !acc);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            reject |= (uint32_t)((rb >> (16 * g)) & 1u) << (cb + g);
            mixed |= (uint32_t)((mb >> (16 * g)) & 1u) << (cb + g);
        }
    }
}

// World corners of the samples [i0, i1] x [j0, j1] x [k0, k1] of lattice g.
__device__ __forceinline__ void box_corners(const fvv_grid& g, int i0, int i1, int j0, int j1,
                                            int k0, int k1, float* lo, float* hi) {
    lo[0] = lattice_coord(g.lo[0] + i0, g.h, g.origin[0]);
    hi[0] = lattice_coord(g.lo[0] + i1, g.h, g.origin[0]);
    lo[1] = lattice_coord(g.lo[1] + j0, g.h, g.origin[1]);
    hi[1] = lattice_coord(g.lo[1] + j1, g.h, g.origin[1]);
    lo[2] = lattice_coord(g.lo[2] + k0, g.h, g.origin[2]);
    hi[2] = lattice_coord(g.lo[2] + k1, g.h, g.origin[2]);
}

// Tile t of lattice g (x fastest, then y, then z): its first sample.
template <int TX>
__device__ __forceinline__ void tile_origin(const fvv_grid& g, uint64_t tile, int& i0, int& j0,
                                            int& k0) {
    constexpr int TY = kBlock / TX;
    const int ntx = (g.dims[0] + TX - 1) / TX;
    const int nty = (g.dims[1] + TY - 1) / TY;
    int bx, by, bz;
    if ((tile >> 32) == 0) {                    // 32-bit index arithmetic where it fits
        const uint32_t t32 = (uint32_t)tile, rq = t32 / (uint32_t)ntx;
        bx = (int)(t32 - rq * (uint32_t)ntx);
        by = (int)(rq % (uint32_t)nty);
        bz = (int)(rq / (uint32_t)nty);
    } else {
        const uint64_t rq = tile / (uint64_t)ntx;
        bx = (int)(tile - rq * (uint64_t)ntx);
        by = (int)(rq % (uint64_t)nty);
        bz = (int)(rq / (uint64_t)nty);
    }
    i0 = bx * TX;
    j0 = by * TY;
    k0 = bz * 4;
}

// ------------------------------------------------------------------ one lattice
template <int TX, int TZ, bool kRows>
__global__ __launch_bounds__(kBlock) void carve_kernel(const CamSet cams,
                                                       const uint32_t* __restrict__ sils,
                                                       const fvv_grid g, uint8_t* __restrict__ occ,
                                                       const RowBits rb) {
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    carve_tile<TX, TZ, kRows ? kBitsLabel : kBitsNone>([&](int c) { return &cams.P[c][0]; },
                              [&](int c) { return sils + c * cam_words; }, cams.n, cams.W, cams.H,
                              cams.wpr, g, blockIdx.x, occ, rb);
}

// Large lattices, most of whose samples lie far from every silhouette, in two
// passes over boxes of 8 x 8 x 4 samples (compact boxes project to small
// rectangles, so more of them are rejected whole than flat tiles of the same
// size): carve_reject_kernel zeroes the occupancy and marks the boxes that no
// camera rejects whole; carve_kept_kernel carves the marked boxes.
constexpr int kRejRows = 16;   // block rows of a rectangle read for a rejection

// Whether the camera cam (P, then the rounding pad) sees no foreground pixel
// in the padded rectangle of the box lo, hi (then no sample of the box is
// occupied), by one lane: the bounds of the 8 corners' quotients, then the
// silhouette's non-empty 8 x 8-pixel blocks under the rectangle (sb: this
// camera's block rows), eight rows at a time until one is non-empty.  A
// rectangle of more than kRejRows block rows or two words of blocks rejects
// nothing.
__device__ __forceinline__ bool cam_rejects_box(const float* cam, int W, int H,
                                                const uint64_t* __restrict__ sb, int bw,
                                                const float* lo, const float* hi) {
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // the (y, z) partial sums, shared by the two corners on x
        const float Y = (k & 1) ? hi[1] : lo[1], Z = (k & 2) ? hi[2] : lo[2];
        const float ayz = __builtin_fmaf(cam[2], Z, __builtin_fmaf(cam[1], Y, cam[3]));
        const float byz = __builtin_fmaf(cam[6], Z, __builtin_fmaf(cam[5], Y, cam[7]));
        const float wyz = __builtin_fmaf(cam[10], Z, __builtin_fmaf(cam[9], Y, cam[11]));
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float X = e ? hi[0] : lo[0];
            const float a = __builtin_fmaf(cam[0], X, ayz);
            const float b = __builtin_fmaf(cam[4], X, byz);
            const float w = __builtin_fmaf(cam[8], X, wyz);
            const float r = __builtin_amdgcn_rcpf(w);
            x0 = fminf(x0, a * r);
            x1 = fmaxf(x1, a * r);
            y0 = fminf(y0, b * r);
            y1 = fmaxf(y1, b * r);
        }
    }
    int cx0, cx1, cy0, cy1;
    bool inside;
    const int st = rect_of_bounds(x0, x1, y0, y1, cam[12], W, H, cx0, cx1, cy0, cy1, inside);
    if (st >= 0)
        return st == kCullReject;
    const int by0 = cy0 >> 3, nby = (cy1 >> 3) - by0 + 1;
    const int bx0 = cx0 >> 3, bx1 = cx1 >> 3, w0 = bx0 >> 6;
    if (nby > kRejRows || (bx1 >> 6) - w0 > 1)
        return false;
    const bool two = (bx1 >> 6) != w0;
    const uint64_t m0 = (~0ull << (bx0 & 63)) & (two ? ~0ull : ~0ull >> (63 - (bx1 & 63)));
    const uint64_t m1 = two ? ~0ull >> (63 - (bx1 & 63)) : 0ull;
    // each batch's loads in bounds and issued at once: rows past the
    // rectangle repeat its last row, the second word repeats the first where
    // there is none
    const uint64_t* row = sb + (int64_t)by0 * bw + w0;
    const int w1 = two ? 1 : 0;
    uint64_t acc = 0ull;
    for (int r0 = 0; r0 < nby && acc == 0ull; r0 += 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint64_t* rr = row + (int64_t)min(r0 + r, nby - 1) * bw;
            acc |= (rr[0] & m0) | (rr[w1] & m1);
        }
    }
    return acc == 0ull;
}

// The boxes of the two-pass carve: nbx x nby x nbz boxes of 8 x 8 x 4 samples,
// x fastest; with the divisions by nbx and nby.
struct RejBoxes {
    uint32_t n, nbx, nby;
    DivU32 by_nbx, by_nby;
};


__device__ __forceinline__ void rej_box_origin(const RejBoxes& bx, uint32_t b, int& i0, int& j0,
                                               int& k0) {
    const uint32_t q = divu32(b, bx.by_nbx), bz = divu32(q, bx.by_nby);
    i0 = 8 * (int)(b - q * bx.nbx);
    j0 = 8 * (int)(q - bz * bx.nby);
    k0 = 4 * (int)bz;
}

// Zeros over the whole occupancy (16-byte stores between the first and the
// last 16-byte boundary), then one thread per (box, camera): a workgroup
// takes per_wg = min(256 / cameras, 64) boxes (cam_of: division by the camera
// count), each camera that rejects a box marks it in LDS, and the
// boxes no camera rejects are appended to list (one atomic on *count per
// workgroup that keeps any; *count is 0 before, order unspecified).
__global__ __launch_bounds__(kBlock) void carve_reject_kernel(const CamSet cams,
                                                              const SilAny sa, const fvv_grid g,
                                                              uint8_t* __restrict__ occ,
                                                              const RejBoxes boxes, int per_wg,
                                                              DivU32 cam_of,
                                                              uint32_t* __restrict__ list,
                                                              uint32_t* __restrict__ count) {
    __shared__ float s_cam[FVV_MAX_CAMS][13];
    __shared__ uint32_t s_rej[kBlock];
    for (int i = threadIdx.x; i < cams.n * 13; i += kBlock) {
        const int c = i / 13, e = i - 13 * c;
        s_cam[c][e] = e < 12 ? cams.P[c][e] : cams.pad[c];
    }
    s_rej[threadIdx.x] = 0u;
    const uint64_t V = (uint64_t)g.dims[0] * (uint64_t)g.dims[1] * (uint64_t)g.dims[2];
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * kBlock;
    const uint64_t mis = (16u - (uint32_t)(reinterpret_cast<uintptr_t>(occ) & 15u)) & 15u;
    const uint64_t head = mis < V ? mis : V;
    const uint64_t n16 = (V - head) >> 4, tail0 = head + (n16 << 4);
    uint4* const body = reinterpret_cast<uint4*>(occ + head);
    for (uint64_t i = tid; i < n16; i += nth)
        body[i] = make_uint4(0u, 0u, 0u, 0u);
    if (tid < head)
        occ[tid] = 0;
    if (tid < V - tail0)
        occ[tail0 + tid] = 0;
    __syncthreads();

    const uint32_t bl = divu32(threadIdx.x, cam_of);
    const int c = (int)(threadIdx.x - bl * (uint32_t)cams.n);
    const uint32_t b = blockIdx.x * (uint32_t)per_wg + bl;
    if (bl < (uint32_t)per_wg && b < boxes.n) {
        int i0, j0, k0;
        rej_box_origin(boxes, b, i0, j0, k0);
        float lo[3], hi[3];
        box_corners(g, i0, min(i0 + 8, g.dims[0]) - 1, j0, min(j0 + 8, g.dims[1]) - 1, k0,
                    min(k0 + 4, g.dims[2]) - 1, lo, hi);
        if (cam_rejects_box(s_cam[c], cams.W, cams.H, sa.bits + (int64_t)c * sa.tph * sa.bw,
                            sa.bw, lo, hi))
            s_rej[bl] = 1u;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {   // per_wg <= 64: the first wave holds every box's flag
        const uint32_t bb = blockIdx.x * (uint32_t)per_wg + threadIdx.x;
        const bool kept = threadIdx.x < (unsigned)per_wg && bb < boxes.n && !s_rej[threadIdx.x];
        const uint64_t km = __ballot(kept);
        if (km) {
            uint32_t at = 0u;
            if (threadIdx.x == 0)
                at = atomicAdd(count, (uint32_t)__popcll(km));
            at = (uint32_t)__builtin_amdgcn_readfirstlane((int)at);
            if (kept)
                list[at + lane_rank(km)] = bb;
        }
    }
}

// One z layer (8 x 8 samples) of a kept box by one wave: lane (x, y) = (l % 8,
// l / 8) holds one sample, tested against 16 cameras at a time in one call
// (cam: matrices and pads in LDS; a camera past the last repeats the last)
// until it is out or the cameras are; then its occupancy byte and, with
// kRows, the labelling's row bits (a box row's 8 bits ORed into its word).
template <bool kRows>
__device__ __forceinline__ void carve_box_layer(const float (*cam)[13],
                                                const uint32_t* __restrict__ sils,
                                                int64_t cam_words, int ncam, int W, int H,
                                                int wpr, const fvv_grid& g, int i0, int j0, int k,
                                                uint8_t* __restrict__ out, const RowBits& rb) {
    const int lane = lane_id();
    const int i = i0 + (lane & 7), j = j0 + (lane >> 3);
    bool alive = i < g.dims[0] && j < g.dims[1] && k < g.dims[2];
    const bool valid = alive;
    const float X = lattice_coord(g.lo[0] + i, g.h, g.origin[0]);
    const float Y = lattice_coord(g.lo[1] + j, g.h, g.origin[1]);
    const float Z = lattice_coord(g.lo[2] + k, g.h, g.origin[2]);
    for (int c0 = 0; c0 < ncam && __ballot(alive) != 0ull; c0 += 16) {
        const float* P[16];
        const uint32_t* S[16];
        float Xs[16], Ys[16], Zs[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = min(c0 + q, ncam - 1);
            P[q] = cam[c];
            S[q] = sils + c * cam_words;
            Xs[q] = X;
            Ys[q] = Y;
            Zs[q] = Z;
        }
        alive = alive && multi_inside<16>(P, Xs, Ys, Zs, S, W, H, wpr) == 0xffffu;
    }
    if (valid)
        out[(uint64_t)k * g.dims[0] * (uint64_t)g.dims[1] + (uint64_t)j * g.dims[0] + i] =
            alive ? 1 : 0;
    if (kRows) {
        const uint64_t bits = (__ballot(alive) >> (8 * (lane >> 3))) & 0xffull;
        if ((lane & 7) == 0 && bits != 0) {
            const int64_t row = (int64_t)j + (int64_t)g.dims[1] * k;
            atomicOr((unsigned long long*)(rb.words + row * rb.wr + (i0 >> 6)),
                     (unsigned long long)(bits << (i0 & 63)));
            atomicOr((unsigned long long*)&rb.rowmask[row >> 6], 1ull << (row & 63));
        }
    }
}

// The kept boxes (list, *count of them): workgroup w of G carves entries w, w +
// G, ... with its four waves, one z layer each; any_bits (any_words words)
// zeroed.
template <bool kRows>
__global__ __launch_bounds__(kBlock) void carve_kept_kernel(const CamSet cams,
                                                            const uint32_t* __restrict__ sils,
                                                            const fvv_grid g,
                                                            uint8_t* __restrict__ occ,
                                                            const RowBits rb,
                                                            const uint32_t* __restrict__ list,
                                                            const uint32_t* __restrict__ count,
                                                            const RejBoxes boxes,
                                                            uint64_t* __restrict__ any_bits,
                                                            int64_t any_words) {
    __shared__ float s_cam[FVV_MAX_CAMS][13];
    for (int i = threadIdx.x; i < cams.n * 13; i += kBlock) {
        const int c = i / 13, e = i - 13 * c;
        s_cam[c][e] = e < 12 ? cams.P[c][e] : cams.pad[c];
    }
    // the non-empty blocks, read by the first pass, cleared for the next frame
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < any_words;
         i += (int64_t)gridDim.x * kBlock)
        any_bits[i] = 0ull;
    __syncthreads();
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t n = min(*count, boxes.n);
    for (uint32_t q = blockIdx.x; q < n; q += gridDim.x) {
        int i0, j0, k0;
        rej_box_origin(boxes, list[q], i0, j0, k0);
        carve_box_layer<kRows>(s_cam, sils, cam_words, cams.n, cams.W, cams.H, cams.wpr, g, i0,
                               j0, k0 + wave, occ, rb);
    }
}

// Camera classification of a whole culled tile (TX x TY x 4 samples from
// i0, j0, k0) by one wave: rejecting and mixed cameras, uniform over the wave.
template <int TX, class Cams>
__device__ __forceinline__ void classify_tile(const Cams& cams, const uint32_t* __restrict__ sils,
                                              const fvv_grid& g, int i0, int j0, int k0,
                                              uint32_t& reject, uint32_t& mixed) {
    constexpr int TY = kBlock / TX;
    float lo[3], hi[3];
    box_corners(g, i0, min(i0 + TX, g.dims[0]) - 1, j0, min(j0 + TY, g.dims[1]) - 1, k0,
                min(k0 + 4, g.dims[2]) - 1, lo, hi);
    classify_box_wave<2>(cams, sils, (int64_t)cams.H * cams.wpr, lo, hi, reject, mixed);
}

// One culled tile (first sample i0, j0, k0).  tile_off (uniform): a camera
// rejects the whole tile, which
// is written as zeros with no other work; tile_mixed: the cameras left to
// classify per sub-block (cameras outside it accept the whole tile).  rb:
// nothing (words null), a fine bitmap (rows of whole words written), or the
// labelling's row bitmap (rowmask set: bits ORed in, rows marked).  Every
// LDS read of a tile happens before its last barrier except the s_occ reads
// of the output pass, and the next tile writes s_occ only after two barriers,
// so consecutive tiles need no barrier between them.
template <int TX, class Cams>
__device__ __forceinline__ void carve_tile_culled(const Cams& cams,
                                                  const uint32_t* __restrict__ sils,
                                                  const fvv_grid& g, int i0, int j0, int k0,
                                                  uint8_t* __restrict__ out, const RowBits& rb,
                                                  bool tile_off = false,
                                                  uint32_t tile_mixed = ~0u) {
    constexpr int TY = kBlock / TX, TZ = 4;
    constexpr int TV = TX * TY * TZ;
    constexpr int SBX = TX / 4;                 // sub-blocks along x (16 in all)
    constexpr int LX = log2_of(TX), LY = log2_of(TY);
    __shared__ uint8_t s_occ[TV];
    __shared__ uint32_t s_mixed[16];
    __shared__ uint32_t s_reject;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    const int tk1 = min(k0 + TZ, g.dims[2]) - 1;
    const int wave = threadIdx.x / kWave, lane = lane_id();

    if (!tile_off) {
        if (threadIdx.x < 16)
            s_mixed[threadIdx.x] = 0;
        if (threadIdx.x == 0)
            s_reject = 0;
        __syncthreads();
        for (int p = threadIdx.x; p < 16 * cams.n; p += kBlock) {
            const int b = p & 15, c = p >> 4;
            const int si0 = i0 + (b % SBX) * 4, sj0 = j0 + (b / SBX) * 4;
            if (si0 >= g.dims[0] || sj0 >= g.dims[1] || !((tile_mixed >> c) & 1u))
                continue;
            float lo[3], hi[3];
            box_corners(g, si0, min(si0 + 4, g.dims[0]) - 1, sj0, min(sj0 + 4, g.dims[1]) - 1,
                        k0, tk1, lo, hi);
            const int cl = classify_box<6, 2>(cams, c, sils + c * cam_words, lo, hi);
            if (cl == kCullReject)
                atomicOr(&s_reject, 1u << b);
            else if (cl == kCullMixed)
                atomicOr(&s_mixed[b], 1u << c);
        }
        __syncthreads();
        // one wave per sub-block, lane = sample (x fastest, then y, then z)
        for (int b = wave; b < 16; b += kBlock / kWave) {
            const int lx = (b % SBX) * 4 + (lane & 3);
            const int ly = (b / SBX) * 4 + ((lane >> 2) & 3);
            const int lz = lane >> 4;
            const bool valid = i0 + lx < g.dims[0] && j0 + ly < g.dims[1] && k0 + lz < g.dims[2];
            bool alive = valid && !((s_reject >> b) & 1u);
            if (__ballot(alive) != 0) {
                const float X = lattice_coord(g.lo[0] + i0 + lx, g.h, g.origin[0]);
                const float Y = lattice_coord(g.lo[1] + j0 + ly, g.h, g.origin[1]);
                const float Z = lattice_coord(g.lo[2] + k0 + lz, g.h, g.origin[2]);
                // wave-uniform: the sub-block's mixed cameras, two per pass
                uint32_t rest = s_mixed[b];
                while (rest && __ballot(alive) != 0) {
                    const int ca = __ffs(rest) - 1;
                    rest &= rest - 1;
                    if (rest) {
                        const int cb = __ffs(rest) - 1;
                        rest &= rest - 1;
                        const float* P2[2] = {cams.Pc(ca), cams.Pc(cb)};
                        const uint32_t* S2[2] = {sils + ca * cam_words,
                                                 sils + cb * cam_words};
                        alive = alive &&
                                group_inside<2>(P2, X, Y, Z, S2, cams.W, cams.H, cams.wpr);
                    } else {
                        const float* P1[1] = {cams.Pc(ca)};
                        const uint32_t* S1[1] = {sils + ca * cam_words};
                        alive = alive &&
                                group_inside<1>(P1, X, Y, Z, S1, cams.W, cams.H, cams.wpr);
                    }
                }
            }
            s_occ[lx + TX * (ly + TY * lz)] = alive ? 1 : 0;
        }
        __syncthreads();
    }
    // output: thread (lx, ly) writes sample row ly, column lx of every z layer
    const uint64_t plane = (uint64_t)g.dims[0] * (uint64_t)g.dims[1];
    const int lx = threadIdx.x & (TX - 1), ly = threadIdx.x >> LX;
    const int i = i0 + lx, j = j0 + ly;
    const bool vxy = i < g.dims[0] && j < g.dims[1];
    uint8_t* const o = out + ((uint64_t)k0 * plane + (uint64_t)j * (uint64_t)g.dims[0] + i);
    if (tile_off && (!rb.words || rb.rowmask)) {   // zeros; a label bitmap gets no bits
        const int nzr = min(TZ, g.dims[2] - k0);
        if (vxy)
            for (int rr = 0; rr < nzr; ++rr)
                o[rr * plane] = 0;
        return;
    }
#pragma unroll
    for (int rr = 0; rr < TZ; ++rr) {
        const int k = k0 + rr;
        const bool valid = vxy && k < g.dims[2];
        const uint8_t bit = tile_off ? 0 : s_occ[rr * kBlock + threadIdx.x];
        if (valid)
            o[rr * plane] = bit;
        // fine bitmap: lanes [TX*q, TX*q + TX) of the wave hold one tile row
        const uint64_t m = __ballot(valid && bit != 0);
        const int q = lane_id() / TX;
        const uint64_t bits = TX == 64 ? m : (m >> (q * TX)) & ((1ull << (TX & 63)) - 1);
        if (rb.words && lx == 0 && j < g.dims[1] && k < g.dims[2]) {
            const int64_t row = (int64_t)j + (int64_t)g.dims[1] * k;
            uint64_t* word = rb.words + row * rb.wr + (i0 >> 6);
            if (rb.rowmask) {
                // the labelling's row bitmap (all-zero before the carve): OR in
                // the set bits and mark the row
                if (bits) {
                    atomicOr((unsigned long long*)word, (unsigned long long)(bits << (i0 & 63)));
                    atomicOr((unsigned long long*)&rb.rowmask[row >> 6], 1ull << (row & 63));
                }
            } else if (TX == 64) {
                *word = bits;
            } else if (TX == 32) {
                reinterpret_cast<uint32_t*>(word)[(i0 >> 5) & 1] = (uint32_t)bits;
            } else {
                reinterpret_cast<uint16_t*>(word)[(i0 >> 4) & 3] = (uint16_t)bits;
            }
        }
    }
}

// One lattice with camera culling (tiles of depth 4): one tile per workgroup,
// the whole-tile classification by the first wave, then the sub-block culling
// of carve_tile_culled.  The camera set's rounding pads must hold over the
// lattice's box (infinite pads leave every camera mixed).
template <int TX>
__global__ __launch_bounds__(kBlock) void carve_culled_kernel(const CamSet cams,
                                                              const uint32_t* __restrict__ sils,
                                                              const fvv_grid g,
                                                              uint8_t* __restrict__ occ,
                                                              const RowBits rb) {
    __shared__ uint32_t s_cls[2];
    int i0, j0, k0;
    tile_origin<TX>(g, blockIdx.x, i0, j0, k0);
    if (threadIdx.x < kWave) {
        uint32_t rej, mix;
        classify_tile<TX>(cams, sils, g, i0, j0, k0, rej, mix);
        if (threadIdx.x == 0) {
            s_cls[0] = rej;
            s_cls[1] = mix;
        }
    }
    __syncthreads();
    const uint32_t rej = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_cls[0]);
    const uint32_t mix = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_cls[1]);
    carve_tile_culled<TX>(cams, sils, g, i0, j0, k0, occ, rb, rej != 0, mix);
}

// Any and all of the pixels [cx0, cx1] x [cy0, cy1] (inside the image) of one
// camera's tiled silhouette tc, when the rectangle lies in at most 2 x 2
// blocks; false (nothing examined) when it spans more.
__device__ __forceinline__ bool rect_any_all_tiled(const uint64_t* __restrict__ tc, int tpr,
                                                   int cx0, int cx1, int cy0, int cy1, bool& any,
                                                   bool& all) {
    const int bx0 = cx0 >> 3, bx1 = cx1 >> 3, by0 = cy0 >> 3, by1 = cy1 >> 3;
    if (bx1 - bx0 > 1 || by1 - by0 > 1)
        return false;
    uint64_t v[4], m[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int bx = bx0 + (d & 1), by = by0 + (d >> 1);
        const bool on = bx <= bx1 && by <= by1;
        // the rectangle's columns and rows within the block (already inside
        // [0, 7] for a block the rectangle touches; clamped for the others)
        const int c0 = min(max(cx0 - 8 * bx, 0), 7), c1 = min(max(cx1 - 8 * bx, 0), 7);
        const int r0 = min(max(cy0 - 8 * by, 0), 7), r1 = min(max(cy1 - 8 * by, 0), 7);
        const uint64_t cols = (uint64_t)((2u << c1) - (1u << c0)) * 0x0101010101010101ull;
        const uint64_t rows = (~0ull >> (8 * (7 - r1))) & (~0ull << (8 * r0));
        m[d] = on ? cols & rows : 0ull;
        v[d] = 0;
        if (on)
            v[d] = tc[(int64_t)by * tpr + bx];
    }
    any = false;
    all = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        any |= (v[d] & m[d]) != 0ull;
        all &= (v[d] & m[d]) == m[d];
    }
    return true;
}

// Classification of one camera for the box of samples with world corners lo,
// hi: reject (no foreground pixel in the padded rectangle), accept (inside the
// image and all foreground) or mixed (also for rectangles of more than 2 x 2
// tiled blocks).  cam: P (12 floats) and the rounding pad.  The corners'
// projection rows are the chains of three fmas in the order z, y, x (the
// rounding pad bounds a chain's error in any order), so the (y, z) partial
// sums are shared by the two corners on x.
__device__ __forceinline__ int classify_box_tiled(const float* cam, int W, int H,
                                                  const uint64_t* __restrict__ tc, int tpr,
                                                  const float* lo, const float* hi) {
    const float pad = cam[12];
    if (!(pad < 1.0f))
        return kCullMixed;
    float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float Y = (k & 1) ? hi[1] : lo[1], Z = (k & 2) ? hi[2] : lo[2];
        const float ayz = __builtin_fmaf(cam[1], Y, __builtin_fmaf(cam[2], Z, cam[3]));
        const float byz = __builtin_fmaf(cam[5], Y, __builtin_fmaf(cam[6], Z, cam[7]));
        const float wyz = __builtin_fmaf(cam[9], Y, __builtin_fmaf(cam[10], Z, cam[11]));
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float X = e ? hi[0] : lo[0];
            const float a = __builtin_fmaf(cam[0], X, ayz);
            const float b = __builtin_fmaf(cam[4], X, byz);
            const float w = __builtin_fmaf(cam[8], X, wyz);
            const float r = __builtin_amdgcn_rcpf(w);
            const float qa = a * r, qb = b * r;
            x0 = fminf(x0, qa);
            x1 = fmaxf(x1, qa);
            y0 = fminf(y0, qb);
            y1 = fmaxf(y1, qb);
        }
    }
    int cx0, cx1, cy0, cy1;
    bool inside;
    const int r0 = rect_of_bounds(x0, x1, y0, y1, pad, W, H, cx0, cx1, cy0, cy1, inside);
    if (r0 >= 0)
        return r0;
    bool any, all;
    if (!rect_any_all_tiled(tc, tpr, cx0, cx1, cy0, cy1, any, all))
        return kCullMixed;
    if (!any)
        return kCullReject;
    return (inside && all) ? kCullAccept : kCullMixed;
}

// The pixel of camera P (12 floats) for the point (X, Y, Z) as the occupancy
// test floors it (sil_test up to the silhouette word): px, py, and whether
// w > 0 and the pixel lies in the W x H image.
__device__ __forceinline__ bool point_pixel_exact(const float* __restrict__ P, float X, float Y,
                                                  float Z, int W, int H, int& px, int& py) {
    const float a = __builtin_fmaf(P[2], Z, __builtin_fmaf(P[1], Y, __builtin_fmaf(P[0], X, P[3])));
    const float b = __builtin_fmaf(P[6], Z, __builtin_fmaf(P[5], Y, __builtin_fmaf(P[4], X, P[7])));
    const float w =
        __builtin_fmaf(P[10], Z, __builtin_fmaf(P[9], Y, __builtin_fmaf(P[8], X, P[11])));
    const float r = __builtin_amdgcn_rcpf(w);
    float qa = a * r, qb = b * r;
    const bool tiny = w > 0.0f && w < 0x1p-64f;
    if (__builtin_expect(__ballot(tiny) != 0, 0)) {
        if (tiny) {
            qa = a / w;
            qb = b / w;
        }
    }
    qa = __builtin_amdgcn_fmed3f(qa, -4.0f, (float)W + 4.0f);
    qb = __builtin_amdgcn_fmed3f(qb, -4.0f, (float)H + 4.0f);
    px = exact_floor(a, w, qa);
    py = exact_floor(b, w, qb);
    return (w > 0.0f) & ((unsigned)px < (unsigned)W) & ((unsigned)py < (unsigned)H);
}

// The pixels of the rectangle [cx0, cx0 + 7] x [cy0, cy0 + 7] of one camera's
// tiled silhouette tc as one 64-bit window, bit 8 r + c = pixel (cx0 + c,
// cy0 + r), from the up to 2 x 2 blocks around its corner (nx, ny: whether the
// rectangle's last column / row, cx1 / cy1, lie in the next block; pixels past
// the image are 0).  Rows are shifted up by cy0 % 8, then each row's pixels
// right by cx0 % 8 with the next block's pixels shifted in.
__device__ __forceinline__ uint64_t tiled_window(const uint64_t* __restrict__ tc, int tpr,
                                                 int cx0, int cy0, bool nx, bool ny, bool on) {
    const uint64_t* tb = tc + (int64_t)(cy0 >> 3) * tpr + (cx0 >> 3);
    uint64_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    if (on)
        b0 = tb[0];
    if (on && nx)
        b1 = tb[1];
    if (on && ny)
        b2 = tb[tpr];
    if (on && nx && ny)
        b3 = tb[tpr + 1];
    const int ox = cx0 & 7, oy = 8 * (cy0 & 7);
    const uint64_t t0 = oy ? (b0 >> oy) | (b2 << (64 - oy)) : b0;
    const uint64_t t1 = oy ? (b1 >> oy) | (b3 << (64 - oy)) : b1;
    const uint64_t lo = (uint64_t)(0xffu >> ox) * 0x0101010101010101ull;
    return ((t0 >> ox) & lo) | (ox ? (t1 << (8 - ox)) & ~lo : 0ull);
}

// A (sub-block, camera) pair's window as the tests read it: the pixels, and
// the window's corner pixel (x | y << 16), or kNoWindow when the camera's
// rectangle is larger than 8 x 8 pixels (its tests then load packed words).
constexpr uint32_t kNoWindow = 0xffffffffu;

struct PairWindow {
    uint64_t bits;
    uint32_t org;
    uint32_t pad_;
};

// One 16 x 4 x 4 block of a fine lattice by one wave (first sample bi0, bj0,
// k0; bi0 is a multiple of 16), without workgroup barriers:
//   1. classification: lane (q, c) = (lane / 16, lane % 16) classifies camera
//      cb + c for the 4 x 4 x 4 sub-block q of the block.  The rectangle
//      [floor(c - r), floor(c + r)] around the rcp quotient c of the
//      sub-block's centre, with the job's radius r for the camera (which
//      bounds how far any point of a 4 x 4 x 4 box moves from its centre's
//      projection, widened by the rounding pad), holds the pixel of every
//      sample of the sub-block.  Clamped to the image: no pixel left -> the
//      camera rejects every sample; otherwise, at most 8 x 8 pixels, the
//      rectangle's pixels as a window from the tiled silhouettes: none set ->
//      reject; all set and the rectangle inside the image -> accept; else
//      mixed, the window kept for the tests.  Larger rectangles are tested
//      from the tiled blocks when they span at most 2 x 2 of them (no
//      window), else count as mixed.
//   2. tests: lane = sample (x, y, z) = (lane % 4, lane / 4 % 4, lane / 16)
//      of each sub-block no camera rejects; each pass tests one mixed camera
//      for each of the four sub-blocks (uniform branches), the pixel's bit
//      read from the pair's window (every in-image sample pixel lies in the
//      clamped rectangle) or, without one, from the packed rows.
//   3. output: the occupancy bytes, and the block's 16 bits of each fine-bitmap
//      row word.
// cam_lds: per camera P and the rounding pad; rho: the job's radii per camera
// (kRhoPer floats); win: this wave's LDS windows [4][FVV_MAX_CAMS].  Returns
// the number of test passes, and in the high half the (sub-block, camera)
// tests they made (wave-uniform counts, for measurement builds).
__device__ __forceinline__ uint32_t carve_block16(const CamSet& cams, const float (*cam_lds)[13],
                                              const float* __restrict__ rho,
                                              PairWindow (*win)[FVV_MAX_CAMS],
                                              const uint32_t* __restrict__ sils,
                                              const uint64_t* __restrict__ tiles, int tpr,
                                              int64_t tpc, const fvv_grid& g, int bi0, int bj0,
                                              int k0, uint8_t* __restrict__ out,
                                              const RowBits& fb) {
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    if (bj0 >= ny)
        return 0u;                                 // no row of the block is in the lattice
    uint32_t n_pass = 0u, n_test = 0u;
    const int lane = lane_id();
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int64_t cam_words = (int64_t)cams.H * cams.wpr;
    uint64_t occ[4] = {0ull, 0ull, 0ull, 0ull};
    if (bi0 < nx) {
        // 1. classification
        const int q = lane >> 4, cl = lane & 15;
        const int si0 = bi0 + 4 * q;
        const bool sb_on = si0 < nx;
        float lo[3], hi[3];
        box_corners(g, min(si0, nx - 1), min(si0 + 3, nx - 1), bj0, min(bj0 + 3, ny - 1), k0,
                    min(k0 + 3, nz - 1), lo, hi);
        const float Xc = 0.5f * (lo[0] + hi[0]), Yc = 0.5f * (lo[1] + hi[1]);
        const float Zc = 0.5f * (lo[2] + hi[2]);
        uint32_t rej[4] = {0u, 0u, 0u, 0u}, mix[4] = {0u, 0u, 0u, 0u};
        for (int cb = 0; cb < cams.n; cb += 16) {
            const int c = cb + cl;
            const bool on = sb_on && c < cams.n;
            const int cc = on ? c : 0;
            const float* P = cam_lds[cc];
            const float rx = rho[cc * kRhoPer + 0], ry = rho[cc * kRhoPer + 1];
            const float a = __builtin_fmaf(P[2], Zc, __builtin_fmaf(P[1], Yc, __builtin_fmaf(P[0], Xc, P[3])));
            const float b = __builtin_fmaf(P[6], Zc, __builtin_fmaf(P[5], Yc, __builtin_fmaf(P[4], Xc, P[7])));
            const float w = __builtin_fmaf(P[10], Zc, __builtin_fmaf(P[9], Yc, __builtin_fmaf(P[8], Xc, P[11])));
            const float r = __builtin_amdgcn_rcpf(w);
            const float W = (float)cams.W, H = (float)cams.H;
            const float qa = __builtin_amdgcn_fmed3f(a * r, -8.0f, W + 8.0f);
            const float qb = __builtin_amdgcn_fmed3f(b * r, -8.0f, H + 8.0f);
            const bool bounded = rx < 64.0f && ry < 64.0f;   // (INFINITY: no bound)
            const int x0 = (int)__builtin_floorf(qa - (bounded ? rx : 0.0f));
            const int x1 = (int)__builtin_floorf(qa + (bounded ? rx : 0.0f));
            const int y0 = (int)__builtin_floorf(qb - (bounded ? ry : 0.0f));
            const int y1 = (int)__builtin_floorf(qb + (bounded ? ry : 0.0f));
            const bool inside = x0 >= 0 && y0 >= 0 && x1 < cams.W && y1 < cams.H;
            const int cx0 = max(x0, 0), cx1 = min(x1, cams.W - 1);
            const int cy0 = max(y0, 0), cy1 = min(y1, cams.H - 1);
            const bool off = cx0 > cx1 || cy0 > cy1;
            const bool small = bounded && !off && cx1 - cx0 <= 7 && cy1 - cy0 <= 7;
            const uint64_t* tc = tiles + cc * tpc;
            const uint64_t wv = tiled_window(tc, tpr, small ? cx0 : 0, small ? cy0 : 0,
                                             (cx1 >> 3) != (cx0 >> 3), (cy1 >> 3) != (cy0 >> 3),
                                             on && small);
            const uint64_t cols = (uint64_t)((2u << (cx1 - cx0 & 7)) - 1u) * 0x0101010101010101ull;
            const uint64_t m = cols & (~0ull >> (8 * (7 - (cy1 - cy0 & 7))));
            bool any = (wv & m) != 0ull, all = (wv & m) == m;
            bool known = small;
            if (__ballot(on && bounded && !off && !small) != 0ull) {
                // rectangles past a window: any / all from the tiled blocks
                bool a2 = false, l2 = true;
                const bool ok2 = on && bounded && !off && !small &&
                                 rect_any_all_tiled(tc, tpr, cx0, cx1, cy0, cy1, a2, l2);
                if (ok2) {
                    any = a2;
                    all = l2;
                    known = true;
                }
            }
            int cls = kCullMixed;
            if (bounded && off)
                cls = kCullReject;
            else if (known)
                cls = !any ? kCullReject : ((inside && all) ? kCullAccept : kCullMixed);
            if (on && cls == kCullMixed) {
                PairWindow pw;
                pw.bits = wv;
                pw.org = small ? ((uint32_t)cx0 | ((uint32_t)cy0 << 16)) : kNoWindow;
                pw.pad_ = 0;
                win[q][c] = pw;
            }
            const uint64_t rb = __ballot(on && cls == kCullReject);
            const uint64_t mb = __ballot(on && cls == kCullMixed);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                rej[s] |= (uint32_t)(rb >> (16 * s)) & 0xffffu;
                mix[s] |= ((uint32_t)(mb >> (16 * s)) & 0xffffu) << cb;
            }
        }
        wave_lds_sync();   // the windows, written above, are read below by every lane
        // 2. tests
        const bool vyz = bj0 + ly < ny && k0 + lz < nz;
        const float Y = lattice_coord(g.lo[1] + bj0 + ly, g.h, g.origin[1]);
        const float Z = lattice_coord(g.lo[2] + k0 + lz, g.h, g.origin[2]);
        float X[4];
        bool alive[4];
        uint32_t rest[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = bi0 + 4 * s + lx;
            X[s] = lattice_coord(g.lo[0] + i, g.h, g.origin[0]);
            alive[s] = vyz && i < nx && rej[s] == 0u;
            rest[s] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(rej[s] == 0u ? mix[s] : 0u));
        }
        while ((rest[0] | rest[1] | rest[2] | rest[3]) != 0u) {
            ++n_pass;
            n_test += (rest[0] != 0u) + (rest[1] != 0u) + (rest[2] != 0u) + (rest[3] != 0u);
            int px[4], py[4];
            bool ok[4], act[4];
            uint32_t word[4], org[4];
            uint64_t wbits[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                act[s] = rest[s] != 0u;
                if (act[s]) {
                    const int c = __ffs(rest[s]) - 1;
                    rest[s] &= rest[s] - 1u;
                    const PairWindow pw = win[s][c];
                    org[s] = (uint32_t)__builtin_amdgcn_readfirstlane((int)pw.org);
                    wbits[s] = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(pw.bits >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pw.bits);
                    ok[s] = point_pixel_exact(cams.Pc(c), X[s], Y, Z, cams.W, cams.H, px[s],
                                              py[s]);
                    word[s] = 0u;
                    if (org[s] == kNoWindow && ok[s])
                        word[s] = sils[c * cam_words + py[s] * cams.wpr + (px[s] >> 5)];
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (act[s]) {
                    bool in;
                    if (org[s] != kNoWindow) {
                        const int ox = (int)(org[s] & 0xffffu), oy = (int)(org[s] >> 16);
                        in = ok[s] && ((wbits[s] >> ((8 * (py[s] - oy) + (px[s] - ox)) & 63)) & 1ull);
                    } else {
                        in = ok[s] && ((word[s] >> (px[s] & 31)) & 1u);
                    }
                    alive[s] = alive[s] && in;
                    if (__ballot(alive[s]) == 0ull)
                        rest[s] = 0u;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
            occ[s] = __ballot(alive[s]);
        wave_lds_sync();   // the next block rewrites the windows
    }
    // 3. output: bytes, lane -> (x, y) = (lane % 16, lane / 16), every z
    const uint64_t plane = (uint64_t)nx * (uint64_t)ny;
    {
        const int x = lane & 15, y = lane >> 4;
        const int i = bi0 + x, j = bj0 + y;
        const int s = x >> 2;
        const uint64_t oq = s == 0 ? occ[0] : s == 1 ? occ[1] : s == 2 ? occ[2] : occ[3];
        if (i < nx && j < ny) {
            uint8_t* o = out + ((uint64_t)k0 * plane + (uint64_t)j * (uint64_t)nx + i);
#pragma unroll
            for (int z = 0; z < 4; ++z)
                if (k0 + z < nz)
                    o[z * plane] = (uint8_t)((oq >> ((x & 3) + 4 * y + 16 * z)) & 1ull);
        }
    }
    // fine bitmap: lane r < 16 -> row (y, z) = (r % 4, r / 4); the block's 16
    // samples along x are bits (bi0 & 63) .. + 15 of the row's word
    if (lane < 16) {
        const int y = lane & 3, z = lane >> 2;
        const int j = bj0 + y, k = k0 + z;
        if (j < ny && k < nz) {
            uint32_t b = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                b |= (uint32_t)((occ[s] >> (4 * y + 16 * z)) & 0xfull) << (4 * s);
            const int64_t row = (int64_t)j + (int64_t)ny * k;
            reinterpret_cast<uint16_t*>(fb.words + row * fb.wr + (bi0 >> 6))[(bi0 & 63) >> 4] =
                (uint16_t)b;
        }
    }
    return n_pass | (n_test << 16);
}

// Measurement builds (FVV_CARVE_PROBE defined) record, for the first
// kProbeWaves waves of the frame's fine carve, the real-time clock (100 MHz)
// at the wave's entry and exit, its block count and the time its workgroup's
// tables took (entry to the barrier after them), and for its first
// kProbeIters blocks their start, end, test passes and tests.
#ifdef FVV_CARVE_PROBE
constexpr int kProbeWaves = 16384, kProbeIters = 4;
__device__ uint64_t carve_probe_blocks[kProbeWaves * kProbeIters][3];
__device__ uint64_t carve_probe_waves[kProbeWaves][3];
#endif

// The fine carve of a frame: the tiles of all carried ROIs dealt out to the
// workgroups in turn (tile t to workgroup t mod grid, then t + grid, ...), so
// every XCD gets an even share of the costly tiles near the surfaces (this
// measured faster than contiguous tile ranges per XCD, which keep each L2's
// share of the silhouettes smaller but leave some XCDs with more work).  A
// workgroup takes whole tiles (TX x TY x 4 samples);
// each of its four waves owns one 16 x 4 x 4 block of the tile (x offset
// 16 (w mod TX/16), y offset 4 (w div TX/16)) and carves it on its own, with
// no workgroup barrier (carve_block16).  Job tables of up to kJobLds ROIs and
// the cameras' matrices and rounding pads are kept in LDS.
constexpr int kJobLds = 64;

template <int TX>
__global__ __launch_bounds__(kBlock, 7) void carve_frame_kernel(const fvv_job* __restrict__ jobs,
                                                             const JobPrefix* __restrict__ pre,
                                                             const uint32_t* __restrict__ counter,
                                                             const CamSet cams,
                                                             const uint32_t* __restrict__ sils,
                                                             const uint64_t* __restrict__ tiles,
                                                             const float* __restrict__ rho,
                                                             uint8_t* __restrict__ out,
                                                             uint64_t* __restrict__ finebits,
                                                             int job_lds, LabelWrite lw) {
    // the workgroups past the carve's write the coarse labels and filtered
    // occupancy and clear the labelling's row bitmap (they start as the
    // carve's tail frees the CUs)
    if (blockIdx.x >= lw.carve_blocks) {
        const int64_t stride = (int64_t)(gridDim.x - lw.carve_blocks) * kBlock;
        const int64_t t0 = (int64_t)(blockIdx.x - lw.carve_blocks) * kBlock + threadIdx.x;
        for (int64_t v = t0; v < lw.V; v += stride)
            label_write_sample(lw, v);
        label_write_clear(lw, t0, stride);
        return;
    }
#ifdef FVV_CARVE_PROBE
    const uint64_t probe_entry = __builtin_amdgcn_s_memrealtime();
    uint32_t probe_blocks = 0;
#endif
    constexpr int BXN = TX / 16;                     // blocks of a tile along x
    __shared__ PairWindow s_win[kBlock / kWave][4][FVV_MAX_CAMS];
    __shared__ uint64_t s_tile_off[kJobLds + 1];
    __shared__ uint64_t s_bit_off[kJobLds];
    __shared__ int64_t s_out[kJobLds];
    __shared__ fvv_grid s_grid[kJobLds];
    __shared__ float s_cam[FVV_MAX_CAMS][13];        // P, then the rounding pad
    // the job tables of the first job_lds jobs (every job the output can hold,
    // up to kJobLds), loaded without waiting for the frame's job count
    for (int j = threadIdx.x; j <= job_lds; j += kBlock) {
        s_tile_off[j] = pre[j].tile_off;
        if (j < job_lds) {
            s_bit_off[j] = pre[j].bit_off;
            s_out[j] = jobs[j].out_offset;
            s_grid[j] = jobs[j].grid;
        }
    }
    const int nj = (int)counter[2];
    const bool lds = nj <= job_lds;
    for (int i = threadIdx.x; i < cams.n * 13; i += kBlock) {
        const int c = i / 13, e = i - 13 * c;
        s_cam[c][e] = e < 12 ? cams.P[c][e] : cams.pad[c];
    }
    __syncthreads();
#ifdef FVV_CARVE_PROBE
    const uint64_t probe_tables = __builtin_amdgcn_s_memrealtime();
#endif
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int xo = 16 * (wave % BXN), yo = 4 * (wave / BXN);
    const int tpr = (cams.W + 7) / 8;
    const int64_t tpc = (int64_t)tpr * ((cams.H + 7) / 8);
    // the tiles' loop, once with the job tables in LDS and once without (two
    // copies, so that neither reads its tables through generic pointers)
    auto tiles_loop = [&](auto in_lds) {
    uint64_t total;
    if constexpr (decltype(in_lds)::value)
        total = s_tile_off[nj];
    else
        total = pre[nj].tile_off;
    const XcdSlice xs{0, total, blockIdx.x, lw.carve_blocks};
    for (uint64_t t = xs.begin + xs.slot; t < xs.end; t += xs.stride) {
        int jb;
        fvv_grid g;
        int64_t out_off;
        uint64_t tile0, bit_off;
        if constexpr (decltype(in_lds)::value) {
            jb = upper_job([&](int m) { return s_tile_off[m]; }, nj, t);
            g = s_grid[jb];
            out_off = s_out[jb];
            tile0 = s_tile_off[jb];
            bit_off = s_bit_off[jb];
        } else {
            jb = upper_job([&](int m) { return pre[m].tile_off; }, nj, t);
            g = jobs[jb].grid;
            out_off = jobs[jb].out_offset;
            tile0 = pre[jb].tile_off;
            bit_off = pre[jb].bit_off;
        }
        RowBits fb{};
        fb.words = finebits + bit_off;
        fb.wr = (g.dims[0] + 63) / 64;
        int i0, j0, k0;
        tile_origin<TX>(g, t - tile0, i0, j0, k0);
#ifdef FVV_CARVE_PROBE
        const uint64_t t_a = __builtin_amdgcn_s_memrealtime();
#endif
        const uint32_t passes_tests =
            carve_block16(cams, s_cam, rho + (int64_t)jb * FVV_MAX_CAMS * kRhoPer, s_win[wave],
                          sils, tiles, tpr, tpc, g, i0 + xo, j0 + yo, k0, out + out_off, fb);
#ifdef FVV_CARVE_PROBE
        const uint64_t t_b = __builtin_amdgcn_s_memrealtime();
        const uint32_t pw = blockIdx.x * (kBlock / kWave) + wave;
        if (lane_id() == 0 && pw < (uint32_t)kProbeWaves && probe_blocks < (uint32_t)kProbeIters) {
            uint64_t* r = carve_probe_blocks[pw * kProbeIters + probe_blocks];
            r[0] = t_a;
            r[1] = t_b;
            r[2] = passes_tests;
        }
        ++probe_blocks;
#else
        (void)passes_tests;
#endif
    }
    };
    if (lds)
        tiles_loop(std::true_type{});
    else
        tiles_loop(std::false_type{});
#ifdef FVV_CARVE_PROBE
    const uint32_t pw = blockIdx.x * (kBlock / kWave) + wave;
    if (lane_id() == 0 && pw < (uint32_t)kProbeWaves) {
        carve_probe_waves[pw][0] = probe_entry;
        carve_probe_waves[pw][1] = __builtin_amdgcn_s_memrealtime();
        // blocks carved, and (high half) the ticks from entry to the tables'
        // barrier
        carve_probe_waves[pw][2] = probe_blocks | ((probe_tables - probe_entry) << 32);
    }
#endif
}

// The batched carve with camera culling: the tile rows (the tiles of one job
// that share y and z, i.e. all its tiles along x) of all jobs in a static
// XCD-aware partition; each job's cameras from the device table and its
// rounding pads from job_pad_kernel.  A workgroup carves whole tile rows, so
// it writes every byte of the TY rows x 4 layers of output samples the row
// covers: each layer's TY sample rows are contiguous in the output, and cache
// lines are written whole by one workgroup (partly written lines are what
// costs HBM write traffic here).  Along the row, each wave classifies one
// tile of a group of four for its whole box (four latency chains of job,
// camera and silhouette loads in flight at once), then the workgroup carves
// the group's tiles one after the other, writing rejected tiles as zeros
// directly.  The tile-row prefix is read from LDS when the job table fits.
constexpr int kBatchedJobLds = 1024;
constexpr int kGroup = kBlock / kWave;
constexpr int kRowRectWords = 8;   // silhouette words per row of a tile row's rectangle

// Zero n bytes from p by the workgroup: 16-byte stores between the first and
// the last 16-byte boundary, byte stores at the ends.
__device__ __forceinline__ void zero_span(uint8_t* p, int64_t n) {
    const int64_t head = (int64_t)((16 - ((uintptr_t)p & 15)) & 15);
    const int64_t h = head < n ? head : n;
    if ((int64_t)threadIdx.x < h)
        p[threadIdx.x] = 0;
    const int64_t n16 = (n - h) / 16;
    uint4* q = reinterpret_cast<uint4*>(p + h);
    for (int64_t i = threadIdx.x; i < n16; i += kBlock)
        q[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t tail0 = h + 16 * n16;
    if ((int64_t)threadIdx.x < n - tail0)
        p[tail0 + threadIdx.x] = 0;
}

template <int TX, bool kLds>
__global__ __launch_bounds__(kBlock, 6) void carve_batched_culled_kernel(
    const fvv_job* __restrict__ jobs, const JobPrefix* __restrict__ pre,
    const uint32_t* __restrict__ counter, const fvv_camera* __restrict__ cams,
    const float* __restrict__ job_pad, const uint32_t* __restrict__ sils,
    uint8_t* __restrict__ out) {
    constexpr int TY = kBlock / TX;
    __shared__ uint64_t s_row_off[kLds ? kBatchedJobLds + 1 : 1];
    __shared__ int32_t s_tile[kGroup][2];      // rejecting, mixed cameras
    const int nj = (int)counter[2];
    if (kLds)
        for (int j = threadIdx.x; j <= nj; j += kBlock)
            s_row_off[j] = pre[j].row_off;
    __syncthreads();
    auto off = [&](int m) -> uint64_t {
        if (kLds)
            return s_row_off[m];
        return pre[m].row_off;
    };
    const XcdSlice xs = xcd_slice(off(nj));
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int jb = 0;
    if (xs.begin + xs.slot < xs.end)
        jb = upper_job(off, nj, xs.begin + xs.slot);
    for (uint64_t row = xs.begin + xs.slot; row < xs.end; row += xs.stride) {
        // rows ascend, so the job index only moves forward
        while (jb + 1 < nj && off(jb + 1) <= row)
            ++jb;
        const int j = __builtin_amdgcn_readfirstlane(jb);
        const fvv_job& job = jobs[j];
        const fvv_grid g = job.grid;
        const JobCams jc{cams + job.cam_base, job_pad + (int64_t)j * FVV_MAX_CAMS, job.n_cams,
                         job.width, job.height, (job.width + 31) / 32};
        const int ntx = (g.dims[0] + TX - 1) / TX;
        const int nty = (g.dims[1] + TY - 1) / TY;
        const uint32_t r = (uint32_t)(row - off(j));
        const int j0 = (int)(r % (uint32_t)nty) * TY, k0 = (int)(r / (uint32_t)nty) * 4;
        // the whole row first: a camera that rejects the row's box rejects
        // every tile of it, and the row's TY x 4 sample rows are written as
        // zeros, each layer's rows one contiguous span
        __syncthreads();                       // the previous row is done with s_tile
        if (wave == 0) {
            float lo[3], hi[3];
            box_corners(g, 0, g.dims[0] - 1, j0, min(j0 + TY, g.dims[1]) - 1, k0,
                        min(k0 + 4, g.dims[2]) - 1, lo, hi);
            uint32_t rej, mix;
            classify_box_wave<kRowRectWords>(jc, sils + job.sil_base, (int64_t)jc.H * jc.wpr, lo, hi,
                                         rej, mix);
            if (lane_id() == 0)
                s_tile[0][0] = (int32_t)rej;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_tile[0][0]) != 0) {
            const int ny = min(j0 + TY, g.dims[1]) - j0;
            const int64_t span = (int64_t)ny * g.dims[0];            // bytes per layer
            const int64_t plane = (int64_t)g.dims[0] * g.dims[1];
            uint8_t* base = out + job.out_offset + (int64_t)j0 * g.dims[0];
            for (int z = 0; z < 4 && k0 + z < g.dims[2]; ++z)
                zero_span(base + (int64_t)(k0 + z) * plane, span);
            continue;
        }
        for (int tx0 = 0; tx0 < ntx; tx0 += kGroup) {
            __syncthreads();                   // the previous group is done with s_tile
            if (tx0 + wave < ntx) {
                uint32_t rej, mix;
                classify_tile<TX>(jc, sils + job.sil_base, g, (tx0 + wave) * TX, j0, k0, rej,
                                  mix);
                if (lane_id() == 0) {
                    s_tile[wave][0] = (int32_t)rej;
                    s_tile[wave][1] = (int32_t)mix;
                }
            }
            __syncthreads();
            for (int w = 0; w < kGroup && tx0 + w < ntx; ++w) {
                // uniform values read back from LDS: scalar registers
                const uint32_t rej = (uint32_t)__builtin_amdgcn_readfirstlane(s_tile[w][0]);
                const uint32_t mix = (uint32_t)__builtin_amdgcn_readfirstlane(s_tile[w][1]);
                carve_tile_culled<TX>(jc, sils + job.sil_base, g, (tx0 + w) * TX, j0, k0,
                                      out + job.out_offset, RowBits{}, rej != 0, mix);
            }
        }
    }
}

hipError_t launch_carve_frame(fvv_ctx* ctx, const fvv_job* jobs, int max_jobs,
                              const CamSet& cams, const uint32_t* sils, const uint64_t* tiles,
                              uint8_t* out, uint64_t* finebits, TileShape t, int blocks,
                              const fvv_grid& coarse, uint8_t* occ_coarse, int32_t* labels,
                              hipStream_t s, hipEvent_t k_start, hipEvent_t k_stop) {
    if (t.tz != 4) {
        // the persistent carve: the events bracket its launch; the labels'
        // write pass goes first
        hipError_t e = launch_label_write(ctx, coarse, occ_coarse, labels, s);
        if (e == hipSuccess && k_start)
            e = hipEventRecord(k_start, s);
        if (e == hipSuccess)
            e = launch_carve_batched(ctx, jobs, 0, ctx->d_cams, sils, out, finebits, t, blocks,
                                     true, s);
        if (e == hipSuccess && k_stop)
            e = hipEventRecord(k_stop, s);
        return e;
    }
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;
    // the coarse labels' write pass rides in the same launch, about eight
    // samples per thread in workgroups after the carve's
    LabelWrite lw = label_write_args(ctx, coarse, occ_coarse, labels);
    lw.carve_blocks = (uint32_t)blocks;
    const int64_t lw_blocks = (lw.V + 8 * kBlock - 1) / (8 * kBlock);
    const int extra = (int)(lw_blocks < 1 ? 1 : (lw_blocks > 4 * ctx->n_cus ? 4 * ctx->n_cus
                                                                              : lw_blocks));
    // jobs: max_jobs entries; the prefix table holds at least max_jobs + 1
    const int job_lds = max_jobs < kJobLds ? max_jobs : kJobLds;
#define X(TXV)                                                                                 \
    if (t.tx == TXV) {                                                                         \
        hipExtLaunchKernelGGL((carve_frame_kernel<TXV>), dim3(blocks + extra), dim3(kBlock), 0, \
                              s, k_start, k_stop, 0, jobs, ctx->d_prefix, ctx->d_counter, cams, \
                              sils, tiles, ctx->d_rho, out, finebits, job_lds, lw);            \
        return hipGetLastError();                                                              \
    }
    X(64) X(32) X(16)
#undef X
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ dispatch
#define FVV_TILE_CASES(X)                                                                  \
    X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(32, 1) X(32, 2) X(32, 4) X(32, 8) X(16, 1)     \
    X(16, 2) X(16, 4) X(16, 8)

hipError_t launch_carve(const CamSet& cams, const uint32_t* sils, const fvv_grid& g, TileShape t,
                        uint8_t* occ, const RowBits* rows, hipStream_t s,
                        const CarveReject* rej) {
    const uint64_t tiles = tiles_of_grid(g, t.tx, t.tz);
    if (tiles == 0)
        return hipSuccess;
    if (tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
    const RowBits rb = rows ? *rows : RowBits{};
    if (t.tz == 4) {                      // camera culling per tile and per 4x4x4 sub-block
#define X(TXV)                                                                                \
        if (t.tx == TXV) {                                                                    \
            hipLaunchKernelGGL((carve_culled_kernel<TXV>), dim3((unsigned)tiles), dim3(kBlock), \
                               0, s, cams, sils, g, occ, rb);                                 \
            return hipGetLastError();                                                         \
        }
        X(64)
        X(32)
        X(16)
#undef X
        return hipErrorInvalidValue;
    }
    const uint64_t V = (uint64_t)g.dims[0] * (uint64_t)g.dims[1] * (uint64_t)g.dims[2];
    if (rej && V >= kRejectMinSamples) {
        RejBoxes boxes;
        boxes.nbx = (uint32_t)((g.dims[0] + 7) / 8);
        boxes.nby = (uint32_t)((g.dims[1] + 7) / 8);
        const uint64_t nb = (uint64_t)boxes.nbx * boxes.nby * (uint64_t)((g.dims[2] + 3) / 4);
        if (nb > 0x7fffffffull)
            return hipErrorInvalidValue;
        boxes.n = (uint32_t)nb;
        boxes.by_nbx = divu32_magic(boxes.nbx);
        boxes.by_nby = divu32_magic(boxes.nby);
        const int per_wg = kBlock / cams.n < kWave ? kBlock / cams.n : kWave;
        const unsigned rblocks = (unsigned)((nb + per_wg - 1) / per_wg);
        hipLaunchKernelGGL(carve_reject_kernel, dim3(rblocks), dim3(kBlock), 0, s, cams, rej->any,
                           g, occ, boxes, per_wg, divu32_magic((uint32_t)cams.n), rej->list,
                           rej->count);
        // four workgroups per CU: every wave of the second pass resident at once
        const unsigned kblocks = (unsigned)rej->n_cus * 4;
        uint64_t* const any_bits = const_cast<uint64_t*>(rej->any.bits);
        const int64_t any_words = (int64_t)cams.n * rej->any.tph * rej->any.bw;
        if (rows)
            hipLaunchKernelGGL(carve_kept_kernel<true>, dim3(kblocks), dim3(kBlock), 0, s, cams,
                               sils, g, occ, rb, rej->list, rej->count, boxes, any_bits,
                               any_words);
        else
            hipLaunchKernelGGL(carve_kept_kernel<false>, dim3(kblocks), dim3(kBlock), 0, s, cams,
                               sils, g, occ, rb, rej->list, rej->count, boxes, any_bits,
                               any_words);
        return hipGetLastError();
    }
#define X(TXV, TZV)                                                                           \
    if (t.tx == TXV && t.tz == TZV) {                                                         \
        if (rows)                                                                             \
            hipLaunchKernelGGL((carve_kernel<TXV, TZV, true>), dim3((unsigned)tiles),         \
                               dim3(kBlock), 0, s, cams, sils, g, occ, rb);                   \
        else                                                                                  \
            hipLaunchKernelGGL((carve_kernel<TXV, TZV, false>), dim3((unsigned)tiles),        \
                               dim3(kBlock), 0, s, cams, sils, g, occ, rb);                   \
        return hipGetLastError();                                                             \
    }
    FVV_TILE_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_carve_batched(fvv_ctx* ctx, const fvv_job* jobs, uint32_t n_jobs,
                                const fvv_camera* cams, const uint32_t* sils, uint8_t* out,
                                uint64_t* finebits, TileShape t, int blocks, bool jobs_prepared,
                                hipStream_t s) {
    // a fresh job table carved without fine bitmaps, 4 samples deep: culled
    if (!jobs_prepared && !finebits && t.tz == 4) {
        blocks = (blocks + kXcds - 1) / kXcds * kXcds;
        const uint64_t pairs = (uint64_t)n_jobs * FVV_MAX_CAMS;
        hipLaunchKernelGGL(job_pad_kernel, dim3((unsigned)((pairs + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, jobs, n_jobs, cams, ctx->d_job_pad);
#define X(TXV)                                                                                 \
        if (t.tx == TXV) {                                                                     \
            hipLaunchKernelGGL((batched_prepare_kernel<TXV, 4>), dim3(1), dim3(kBlock), 0, s,  \
                               jobs, n_jobs, ctx->d_prefix, ctx->d_counter, ctx->d_status,     \
                               (uint32_t)blocks);                                              \
            if (n_jobs <= (uint32_t)kBatchedJobLds)                                           \
                hipLaunchKernelGGL((carve_batched_culled_kernel<TXV, true>), dim3(blocks),     \
                                   dim3(kBlock), 0, s, jobs, ctx->d_prefix, ctx->d_counter,    \
                                   cams, ctx->d_job_pad, sils, out);                           \
            else                                                                               \
                hipLaunchKernelGGL((carve_batched_culled_kernel<TXV, false>), dim3(blocks),    \
                                   dim3(kBlock), 0, s, jobs, ctx->d_prefix, ctx->d_counter,    \
                                   cams, ctx->d_job_pad, sils, out);                           \
            return hipGetLastError();                                                          \
        }
        X(64) X(32) X(16)
#undef X
        return hipErrorInvalidValue;
    }
#define X(TXV, TZV)                                                                             \
    if (t.tx == TXV && t.tz == TZV) {                                                           \
        if (!jobs_prepared)                                                                     \
            hipLaunchKernelGGL((batched_prepare_kernel<TXV, TZV>), dim3(1), dim3(kBlock), 0, s,  \
                               jobs, n_jobs, ctx->d_prefix, ctx->d_counter, ctx->d_status,       \
                               (uint32_t)blocks);                                               \
        if (finebits)                                                                           \
            hipLaunchKernelGGL((carve_persistent_kernel<TXV, TZV, true>), dim3(blocks),          \
                               dim3(kBlock), 0, s, jobs, ctx->d_prefix, ctx->d_counter, cams,    \
                               sils, out, finebits);                                            \
        else                                                                                    \
            hipLaunchKernelGGL((carve_persistent_kernel<TXV, TZV, false>), dim3(blocks),         \
                               dim3(kBlock), 0, s, jobs, ctx->d_prefix, ctx->d_counter, cams,    \
                               sils, out, finebits);                                            \
        return hipGetLastError();                                                               \
    }
    FVV_TILE_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace fvv

#ifdef FVV_CARVE_PROBE
// Measurement builds only: the fine carve's probe tables to host memory
// (blocks: kProbeWaves * kProbeIters * 3 words, waves: kProbeWaves * 3), and
// their clearing before a run.
extern "C" int32_t fvv_carve_probe_read(uint64_t* blocks, uint64_t* waves) {
    if (!blocks || !waves)
        return FVV_EINVAL;
    hipError_t e = hipMemcpyFromSymbol(blocks, HIP_SYMBOL(fvv::carve_probe_blocks),
                                       sizeof(fvv::carve_probe_blocks));
    if (e == hipSuccess)
        e = hipMemcpyFromSymbol(waves, HIP_SYMBOL(fvv::carve_probe_waves),
                                sizeof(fvv::carve_probe_waves));
    return e == hipSuccess ? FVV_OK : FVV_EDEVICE;
}

extern "C" int32_t fvv_carve_probe_clear() {
    void* b = nullptr;
    void* w = nullptr;
    hipError_t e = hipGetSymbolAddress(&b, HIP_SYMBOL(fvv::carve_probe_blocks));
    if (e == hipSuccess)
        e = hipGetSymbolAddress(&w, HIP_SYMBOL(fvv::carve_probe_waves));
    if (e == hipSuccess)
        e = hipMemset(b, 0, sizeof(fvv::carve_probe_blocks));
    if (e == hipSuccess)
        e = hipMemset(w, 0, sizeof(fvv::carve_probe_waves));
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    return e == hipSuccess ? FVV_OK : FVV_EDEVICE;
}
#endif
