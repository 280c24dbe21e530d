// What the blend kernels share: the cell layout of a tile, the exact cull
// of a staged Gaussian against the cells, and the bit transpose that turns
// per-Gaussian cell masks into per-cell walk masks.
//
// Layout: a tile of TW x TH pixels is cut into cells of CW x CH pixels, one
// cell per lane, numbered row-major over the tile; a wave owns 64
// consecutive cells (whole cell rows).  Every lane walks, in list order, only
// the staged Gaussians whose support (alpha >= 1/255, section 3's skip rule)
// reaches a pixel centre of its cell, so the lanes of a wave walk different
// Gaussians in the same instructions.
#pragma once

#include "gs_device.h"

namespace gs {

template <int TW_, int TH_, int CW_, int CH_>
struct Cells {
    static constexpr int TW = TW_, TH = TH_, CW = CW_, CH = CH_;
    static constexpr int NT = TW * TH;            // pixels of the tile
    static constexpr int CPR = TW / CW;           // cells per row
    static constexpr int NCELL = CPR * (TH / CH);
    static constexpr int WAVES = NCELL / kWave;   // waves of a workgroup
    static constexpr int NP = CW * CH;            // pixels per lane
    static constexpr int ROWS_W = kWave / CPR;    // cell rows per wave
    static constexpr int PXROWS_W = ROWS_W * CH;  // pixel rows per wave
    static constexpr int CW_SHIFT = CW == 2 ? 1 : 0;
    static_assert(NCELL % kWave == 0 && kWave % CPR == 0, "cell layout");
    static_assert(CW <= 2 && CH <= 2 && CPR <= 16, "cell layout");
};

// The cell layout used for each supported tile shape: 2x2 cells, except
// 8x8 tiles (1x1, 64 lanes) and 16x8 tiles (2x1, 64 lanes).
template <int TW, int TH> struct CellsFor { using L = Cells<TW, TH, 2, 2>; };
template <> struct CellsFor<8, 8> { using L = Cells<8, 8, 1, 1>; };
template <> struct CellsFor<16, 8> { using L = Cells<16, 8, 2, 1>; };

// The forward's layout.  It has no per-entry reduction, so on 16x16 tiles
// it walks 2x1 cells (two waves) where the backward walks 2x2: fewer
// evaluations of pixels outside the support (35.7M instead of 42.3M on the
// 1M-Gaussian 1080p view) for little more bookkeeping, 120 -> 112 us.  The
// backward keeps 2x2 cells, where narrower cells cost more slots and
// combine work than they save (236 -> 305 us with 2x1); the forward writes
// the cell masks it keeps in the backward's layout (keep_mask in
// render_fwd.hip).  On 32-wide tiles (four waves and more with 2x1 cells)
// the narrower forward measured no faster (batched cells at 32x16: 5.03 ->
// 5.11 ms), so they keep one layout.
template <int TW, int TH> struct FwdCellsFor { using L = typename CellsFor<TW, TH>::L; };
template <> struct FwdCellsFor<16, 16> { using L = Cells<16, 16, 2, 1>; };

// 64-bit mask of the cells of one wave that a staged Gaussian can reach:
// bit c is set when some pixel centre of cell c (c = row * CPR + column
// within the wave's cells) may have alpha >= 1/255.  For each pixel row
// of the wave the support is the chord of the ellipse
//   ca dx^2 + cb dx dy + cc dy^2 >= thr
// (base-2 exponent of the Gaussian, thr = -log2(255 o); ca, cc < 0) at the
// row's centre height: with dy fixed the exponent is a concave quadratic in
// dx, whose roots bound the chord.  Its discriminant is quadratic in dy,
// (cb^2 - 4 ca cc) dy^2 + 4 ca thr, and its centre linear, -cb dy / (2 ca),
// with coefficients fixed per Gaussian.  The threshold is lowered by a
// margin (2e-3 + 2e-4 |thr| in base-2 units, far above the FP32 error of
// the exponent the blend evaluates) and the chord widened by 1e-3 px, so
// every pixel the blend can find at or above 1/255 is covered; the chords
// of a cell row's pixel rows are merged into one interval before they are
// turned into cells (a superset: covering a few more only costs
// evaluations that the blend then skips).  x0: the tile's first pixel
// column, y0: the wave's first pixel row (image coordinates).
template <class L>
__device__ __forceinline__ uint64_t cell_mask(const Staged& g, int x0, int y0) {
    const float ca = g.coef.x, cb = g.coef.y, cc = g.coef.z;
    const float thm = g.col.w - (2e-3f + 2e-4f * fabsf(g.col.w));
    const float ia = 0.5f * __builtin_amdgcn_rcpf(ca);        // 1 / (2 ca) < 0
    const float k2 = __builtin_fmaf(cb, cb, (-4.0f * ca) * cc);  // discriminant = k2 dy^2 + k0
    const float k0 = (4.0f * ca) * thm;
    const float m1 = -cb * ia;                                   // chord centre = m1 dy (offset units)
    // pixel column p (tile-local) has offset dx = p - xs from the centre;
    // the chord's ends are widened by 1e-3 px
    const float xs = ((g.geo.x - (float)x0) + g.geo.y) - 0.5f;
    const float xs_lo = xs - 1e-3f, xs_hi = xs + 1e-3f;
    uint32_t lo = 0u, hi = 0u;
#pragma unroll
    for (int r = 0; r < L::ROWS_W; ++r) {
        float cl = __builtin_inff(), ch = -__builtin_inff();   // merged chord of the cell row
#pragma unroll
        for (int q = 0; q < L::CH; ++q) {
            const int j = r * L::CH + q;
            const float dy = (((float)(y0 + j) + 0.5f) - g.geo.z) - g.geo.w;
            const float D = __builtin_fmaf(k2, dy * dy, k0);
            const float s = __builtin_amdgcn_sqrtf(fmaxf(D, 0.0f));   // ~1 ulp, covered by the margins
            const float plo = __builtin_fmaf(s, ia, __builtin_fmaf(m1, dy, xs_lo));
            const float phi = __builtin_fmaf(-s, ia, __builtin_fmaf(m1, dy, xs_hi));
            cl = D >= 0.0f ? fminf(cl, plo) : cl;
            ch = D >= 0.0f ? fmaxf(ch, phi) : ch;
        }
        // covered pixel columns, clamped to the tile before the conversion
        const int c0 = (int)__builtin_ceilf(fminf(fmaxf(cl, -1.0f), (float)L::TW));
        const int c1 = (int)__builtin_floorf(fminf(fmaxf(ch, -1.0f), (float)L::TW));
        const bool ok = (c0 <= c1) & (c1 >= 0) & (c0 < L::TW);
        const int a0 = max(c0, 0) >> L::CW_SHIFT, a1 = min(c1, L::TW - 1) >> L::CW_SHIFT;
        const uint32_t bits = ok ? ((2u << a1) - (1u << a0)) : 0u;
        const int sh = r * L::CPR;                               // the row's cells within the 64 bits
        if (sh < 32) lo |= bits << sh;
        else hi |= bits << (sh - 32);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Transpose of a 64 x 64 bit matrix held one row per lane: on entry lane k
// holds row k (bit c = element (k, c)), on return lane c holds column c (bit
// k = element (k, c)).  Recursive block swap: at each size s the lanes k and
// k ^ s exchange the off-diagonal s x s blocks.  Must be called by all 64
// lanes of the wave.
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {   // s = 32: the lower lanes take the partner's low word as their high word
        const bool up = (lane & 32) != 0;
        const uint32_t r = xor_lane(up ? lo : hi, 32);
        if (up) lo = r;
        else hi = r;
    }
#define GS_TSTAGE(S, M0)                                                       \
    {                                                                          \
        const bool up = (lane & (S)) != 0;                                     \
        const uint32_t keep = up ? ~(uint32_t)(M0) : (uint32_t)(M0);           \
        const uint32_t rl = xor_lane(lo & ~keep, (S)), rh = xor_lane(hi & ~keep, (S)); \
        lo = (lo & keep) | (up ? (rl >> (S)) : (rl << (S)));                   \
        hi = (hi & keep) | (up ? (rh >> (S)) : (rh << (S)));                   \
    }
    GS_TSTAGE(16, 0x0000FFFFu)
    GS_TSTAGE(8, 0x00FF00FFu)
    GS_TSTAGE(4, 0x0F0F0F0Fu)
    GS_TSTAGE(2, 0x33333333u)
    GS_TSTAGE(1, 0x55555555u)
#undef GS_TSTAGE
    return ((uint64_t)hi << 32) | lo;
}

// The staged record `k` (k < 1024) of an LDS array; the bound lets the byte
// offset 48 k use the full-rate 24-bit multiply.
__device__ __forceinline__ const Staged& staged_at(const Staged* s, int k) {
    static_assert(sizeof(Staged) == 48, "staged record layout");
    return *reinterpret_cast<const Staged*>(reinterpret_cast<const char*>(s) + ((unsigned)k & 0x3FFu) * 48u);
}

// Staged records as three arrays (the forward's batches): entry k's
// values sit at 16 k in each, so its address is a shift where the 48-byte
// records of an array of Staged take a multiply (a quarter-rate 32-bit one
// where the compiler cannot bound k).
template <int B>
struct StagedSoA {
    float4 geo[B], coef[B], col[B];
    __device__ __forceinline__ void put(int j, const Staged& g) {
        geo[j] = g.geo;
        coef[j] = g.coef;
        col[j] = g.col;
    }
    __device__ __forceinline__ Staged get(int k) const {
        Staged g;
        g.geo = geo[k];
        g.coef = coef[k];
        g.col = col[k];
        return g;
    }
};

// Stage list entries b0 + j (j < nb <= PER * nthreads) of a tile into
// LDS: each thread issues all of its value loads, then all of its record
// loads, before the first wait, so a batch costs two memory latencies.
template <int PER>
__device__ __forceinline__ void stage_batch(Staged* s, const Rec* __restrict__ rec, const uint32_t* __restrict__ vals,
                                            uint32_t b0, int nb, int tid, int nthreads, uint32_t* gid_out = nullptr) {
    uint32_t v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * nthreads;
        v[q] = j < nb ? vals[b0 + (uint32_t)j] : 0u;
    }
    Rec r[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (tid + q * nthreads < nb) r[q] = rec[v[q]];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * nthreads;
        if (j < nb) {
            s[j] = stage_rec(r[q]);
            if (gid_out) gid_out[j] = v[q];
        }
    }
}

// The same into three arrays.
template <int PER, int B>
__device__ __forceinline__ void stage_batch(StagedSoA<B>& s, const Rec* __restrict__ rec,
                                            const uint32_t* __restrict__ vals, uint32_t b0, int nb, int tid,
                                            int nthreads) {
    uint32_t v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * nthreads;
        v[q] = j < nb ? vals[b0 + (uint32_t)j] : 0u;
    }
    Rec r[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (tid + q * nthreads < nb) r[q] = rec[v[q]];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = tid + q * nthreads;
        if (j < nb) s.put(j, stage_rec(r[q]));
    }
}

// Index of the lowest / highest set bit of a non-zero 64-bit mask.
__device__ __forceinline__ int low_bit(uint64_t m) { return (int)__builtin_ctzll(m); }
__device__ __forceinline__ int high_bit(uint64_t m) { return 63 - (int)__builtin_clzll(m); }

}  // namespace gs
