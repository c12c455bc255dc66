// Body of the fused red/black Metropolis sweep for gfx950 (Sec. 2.2.2 single checkerboard, block temperatures),
// shared by the single-scene kernel (sweep.hip) and the batched persistent kernel (batched.hip).
//
// One call = one sweep k of one 64 x FTH tile for a chunk of realizations.  The state is double-buffered: the tile
// reads sweep k-1 from `src` and writes sweep k to `dst`, so it may read its neighbours' cells while they are being
// updated elsewhere.
//
// Staged once per call: the sample cells of the tile and a two-site ring (their angles and (cos, sin) never
// change), the temperature of every block the region touches, the compacted lists of pairs to update, the list of
// colour-1 sample sites that border a gap, and the energy of the bonds that only join samples.
//
// Per realization:
//   1. the gap cells of the region arrive from registers (loaded during the previous realization) and get their
//      (cos, sin) of 2 pi q t; the next realization's gap cells are then requested into registers;
//   2. colour 0 is updated on the tile and on the one-site ring around it: a ring site's update uses the same
//      counter-based random numbers and the same neighbours as in the tile that owns it, so it is bit-identical;
//   3. colour 1 is updated on the tile (its colour-0 neighbours, ring included, are now current); the energy of the
//      bonds of each updated colour-1 site is taken from the local field just computed;
//   4. the bonds of colour-1 sample sites that touch a gap are added (each bond has exactly one colour-1 end, so
//      the tiles together count every bond once), and the gap cells of the tile are written to `dst`.
//
// LDS layout: per colour, per row, the cells of that colour are contiguous ("colour-split"), so the neighbourhood
// of a same-colour pair is five vector LDS reads.  A cell's angle is stored negated (sign bit set, -0 for 0) when it
// is a sample or lies outside the grid: such cells are never updated; a cell outside the grid also keeps
// (cos, sin) = (0, 0), which no angle has, so a neighbour is present exactly when its (cos, sin) is not zero.
//
// Update lists.  The common case (every temperature block the region touches fits the LDS table, and block columns
// are whole groups of four columns, so both sites of a pair share a block) uses 16-bit codes: the LDS index of the
// lowest cell a site or pair reads, and the table index of its block.  Pairs with both sites free grow from the
// front of each colour's list; pairs with one free site are listed as that site, from the back.  Row, pair index,
// column parity and the random-stream counter follow from the LDS index with full-rate 24-bit arithmetic, and the
// five neighbourhood reads are immediate offsets from it.  Other block shapes take the generic path, whose codes
// hold row, pair and site mask.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "metropolis.hpp"

namespace mpr {

template <int FTH>
struct Tile {
    static constexpr int FT_W = 64, FT_H = FTH, FS_NT = 256;
    static constexpr int RH = FT_H + 4;          // LDS rows: tile rows plus two above and two below
    static constexpr int RW = FT_W + 4;          // region columns: tile plus two on each side
    static constexpr int CW = 40;                // LDS cells per colour per row (34 used, 3 leading, 3 trailing pads)
    static constexpr int NPR = FT_W / 4 + 2;     // pairs per row touching the tile or its one-site ring (0 .. 17)
    static constexpr int MAX_RED = (FT_H + 2) * NPR;
    static constexpr int MAX_BLK = FT_H * (FT_W / 4);
    static constexpr int MAX_EOBS = FT_H * (FT_W / 2);
    // Region cells per thread: the 64 middle columns are walked by lane (tid & 63) on rows (tid >> 6) + 4k,
    // k < RH / 4; the four side columns (0, 1, 66, 67) of the RH rows by threads 0 .. 4 RH - 1, one each.
    static constexpr int MAIN_K = RH / 4;
    static constexpr int CPT = MAIN_K + 1;
    static constexpr int TP_CAP = 32;            // temperature blocks a region may touch for the LDS table
    static constexpr int CS_ROW2 = CW;           // float2 cells per LDS row of one colour
    static constexpr int CS_COL2 = RH * CW;      // float2 cells per colour
    static_assert(CW == 40, "the row division of the fast-path codes assumes 40 cells per colour and row");
    static_assert(RH * CW <= 2048, "fast-path codes hold 11-bit LDS indices of colour-0 cells");
    static_assert(RH % 4 == 0 && 4 * RH <= FS_NT, "cell walk assumes RH % 4 == 0 and 4 RH <= 256");
};

template <int FTH>
struct alignas(16) LdsT {
    using C = Tile<FTH>;
    float2 cs[2][C::RH][C::CW];               // (cos, sin) of 2 pi q t, per colour
    float t[2][C::RH][C::CW];                 // angles per colour; negative (or -0) = sample / outside the grid
    int brow[C::RH];                          // temperature-block row offset per LDS row
    int bcol[C::RW];                          // temperature-block column per region column
    TBand tp[C::TP_CAP];                      // temperatures of the blocks the region touches
    uint16_t items[C::MAX_RED + C::MAX_BLK];  // colour-0 list, then colour-1 list (fast or generic codes)
    uint16_t eobs[C::MAX_EOBS];               // colour-1 sample sites of the tile with a gap neighbour: row << 8 | J
    int wcnt[2][C::FS_NT / 64];
    long long red[C::FS_NT / 64];
};

__device__ __forceinline__ int cell_J(int xl) { return (xl >> 1) + 3; }

// Energies are summed as fixed-point integers: a site's bond energy / J (at most 4 in magnitude) in units of 2^-24,
// an int32, summed exactly (a thread's sites stay below 2^30; int64 across threads).  Integer sums do not depend on
// their order, so the energy series (and the stopping decision) does not depend on the tiling, the realization
// chunks or batching.
__device__ __forceinline__ int to_fix(float x) { return __float2int_rn(x * 16777216.0f); }
__device__ __forceinline__ bool is_fixed(float t) { return __float_as_uint(t) >> 31; }
__device__ __forceinline__ bool present(float2 cs) { return cs.x != 0.0f || cs.y != 0.0f; }

// Appends `val` to list[base ...] for the threads with `flag`, in thread order; every thread must call it.
__device__ __forceinline__ int compact(bool flag, uint16_t val, uint16_t* list, int base, int* wcnt)
{
    const uint64_t bal = __ballot(flag);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) wcnt[wid] = __popcll(bal);
    __syncthreads();
    int off = base, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wid) off += wcnt[w];
        tot += wcnt[w];
    }
    if (flag) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = val;
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(base + tot);     // uniform: keep list lengths in scalar registers
}

// Two-ended append: category 1 to the front of list[0 .. cap), category 2 to the back (list[cap - 1 - k]), each in
// thread order; every thread must call it.  nf / nh count the entries at the front / back.
__device__ __forceinline__ void compact2(int cat, uint16_t val, uint16_t* list, int cap, int& nf, int& nh,
                                         int (*wcnt)[4])
{
    const uint64_t bf = __ballot(cat == 1), bh = __ballot(cat == 2);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        wcnt[0][wid] = __popcll(bf);
        wcnt[1][wid] = __popcll(bh);
    }
    __syncthreads();
    int of = nf, oh = nh, tf = 0, th = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wid) {
            of += wcnt[0][w];
            oh += wcnt[1][w];
        }
        tf += wcnt[0][w];
        th += wcnt[1][w];
    }
    const uint64_t below = (1ull << lane) - 1ull;
    if (cat == 1) list[of + __popcll(bf & below)] = val;
    else if (cat == 2) list[cap - 1 - (oh + __popcll(bh & below))] = val;
    __syncthreads();
    nf = __builtin_amdgcn_readfirstlane(nf + tf);
    nh = __builtin_amdgcn_readfirstlane(nh + th);
}

// One Metropolis update from the LDS neighbourhood: own (cos, sin) o, neighbours up u, left l, right rt, down d,
// proposal / acceptance words wp / wa, block temperature tb.  The index arguments are LDS cell indices (the t and
// cs arrays share them) of the site and of its neighbours, read only on the exact path.  Returns the energy / J of
// the site's bonds after the update (fixed point) when ENERGY.
template <int FTH, bool ENERGY>
__device__ __forceinline__ int site_update(LdsT<FTH>& L, const SweepFusedArgs& a, float2 o, float2 u, float2 l,
                                                 float2 rt, float2 d, uint32_t wp, uint32_t wa, const TBand& tb,
                                                 int i_own, int i_u, int i_l, int i_r, int i_d)
{
    float* const t = &L.t[0][0][0];
    float2* const cs = &L.cs[0][0][0];
    const float Cx = ((u.x + l.x) + rt.x) + d.x;
    const float Sy = ((u.y + l.y) + rt.y) + d.y;
    const float tp = u24(wp);
    const float ui = (float)(wa >> 8);                 // u2 = ui 2^-24
    const float ang = a.q * tp;
    const float cp = cos_rev(ang), sp = sin_rev(ang);
    const float X = fmaf(cp - o.x, Cx, (sp - o.y) * Sy);    // dE = -J X
    int dec = filter32(X, ui, tb, a.J, a.delta_e);
    if (dec < 0) {
        const unsigned pres = (present(u) ? 1u : 0u) | (present(l) ? 2u : 0u) | (present(rt) ? 4u : 0u) |
                              (present(d) ? 8u : 0u);
        dec = exact64(tp, t[i_own], fabsf(t[i_u]), fabsf(t[i_l]), fabsf(t[i_r]), fabsf(t[i_d]), pres, a.two_pi_q,
                      a.Jd, tb.T, ui * 5.9604644775390625e-8f)
                  ? 1
                  : 0;
    }
    float cf = o.x, sf = o.y;
    if (dec) {
        t[i_own] = tp;
        cs[i_own] = make_float2(cp, sp);
        cf = cp;
        sf = sp;
    }
    return ENERGY ? to_fix(-fmaf(cf, Cx, sf * Sy)) : 0;
}

// Fast-path offsets, in LDS cells (float2 units) from the lowest cell a colour-COLOUR pair reads: the pair itself,
// the other colour's cells above and below, and the other colour's cells in the same row.
template <int FTH, int COLOUR>
struct FastOff {
    using C = Tile<FTH>;
    static constexpr int OWN = COLOUR == 0 ? 0 : C::CS_COL2 + C::CW;
    static constexpr int UP = COLOUR == 0 ? C::CS_COL2 - C::CW : 0;
    static constexpr int DN = COLOUR == 0 ? C::CS_COL2 + C::CW : 2 * C::CW;
    static constexpr int MID = COLOUR == 0 ? C::CS_COL2 : C::CW;
};

// Fast-path update of one colour: full pairs list[0 .. nf), single sites list[cap - nh .. cap).  `ctr_base` is the
// colour's random-stream counter offset (see the list builder).
template <int FTH, int COLOUR, bool ENERGY>
__device__ __forceinline__ int fast_colour(LdsT<FTH>& L, const SweepFusedArgs& a, const uint16_t* list,
                                                 int cap, int nf, int nh, uint32_t ctr_base, uint32_t r_global,
                                                 int tid)
{
    using O = FastOff<FTH, COLOUR>;
    const uint32_t w3 = ctr_word3(a.scene, TAG_SWEEP, (uint32_t)COLOUR);
    const int mw20 = a.Mw - 20;
    const float2* const cs = &L.cs[0][0][0];
    int e_sum = 0;
    // Software-pipelined: the next item's code is read one iteration ahead, and the neighbourhood reads are issued
    // before the Philox rounds (the empty asm keeps them there), so their LDS latency is covered by the rounds.
    constexpr int NT = Tile<FTH>::FS_NT;
    int v = tid;
    unsigned code_next = list[v < nf ? v : 0];
    for (; v < nf; v += NT) {
        const unsigned code = code_next;
        code_next = list[v + NT < nf ? v + NT : 0];         // (a valid index either way: no branch)
        const int a4 = (int)(code & 2047u);
        const int q = (int)(__umul24((unsigned)a4, 3277u) >> 16);     // a4 / 20: the LDS row (minus one for colour 1)
        const int delta = q & 1;
        const int b = 2 * a4;
        const int hb = b + O::MID + delta;
        const TBand tb = L.tp[code >> 11];
        const float4 own = *reinterpret_cast<const float4*>(&cs[b + O::OWN]);
        const float4 up = *reinterpret_cast<const float4*>(&cs[b + O::UP]);
        const float4 dn = *reinterpret_cast<const float4*>(&cs[b + O::DN]);
        const float2 x0 = cs[hb - 1], x1 = cs[hb], x2 = cs[hb + 1];
        asm volatile("" ::: "memory");
        const uint32_t c0 = (uint32_t)__mul24(q, mw20) + (uint32_t)a4 + ctr_base;
        const U4 w = philox_x3(c0, a.sweep, r_global, w3, a.key0, a.key1);
        e_sum += site_update<FTH, ENERGY>(L, a, make_float2(own.x, own.y), make_float2(up.x, up.y), x0, x1,
                                          make_float2(dn.x, dn.y), w.x, w.y, tb, b + O::OWN, b + O::UP, hb - 1, hb,
                                          b + O::DN);
        e_sum += site_update<FTH, ENERGY>(L, a, make_float2(own.z, own.w), make_float2(up.z, up.w), x1, x2,
                                          make_float2(dn.z, dn.w), w.z, w.w, tb, b + 1 + O::OWN, b + 1 + O::UP, hb,
                                          hb + 1, b + 1 + O::DN);
    }
    const uint16_t* const half = list + (cap - nh);
    code_next = half[v < nf + nh ? v - nf : 0];
    for (; v < nf + nh; v += NT) {
        const unsigned code = code_next;
        code_next = half[v + NT < nf + nh ? v + NT - nf : 0];
        const int s2 = (int)(code & 2047u);
        const int a4 = s2 >> 1, h = s2 & 1;
        const int q = (int)(__umul24((unsigned)s2, 3277u) >> 17);     // s2 / 40
        const int delta = q & 1;
        const int hb = s2 + O::MID + delta;
        const TBand tb = L.tp[code >> 11];
        const float2 o = cs[s2 + O::OWN], u = cs[s2 + O::UP], d = cs[s2 + O::DN], l = cs[hb - 1], rt = cs[hb];
        asm volatile("" ::: "memory");
        const uint32_t c0 = (uint32_t)__mul24(q, mw20) + (uint32_t)a4 + ctr_base;
        const U4 w = philox_x3(c0, a.sweep, r_global, w3, a.key0, a.key1);
        e_sum += site_update<FTH, ENERGY>(L, a, o, u, l, rt, d, h ? w.z : w.x, h ? w.w : w.y, tb, s2 + O::OWN,
                                          s2 + O::UP, hb - 1, hb, s2 + O::DN);
    }
    return e_sum;
}

// Generic update of the listed pairs of one colour (codes row << 8 | pair << 2 | site mask), for the block shapes
// the fast lists do not cover; block temperatures are read from global memory (brow / bcol hold global offsets).
template <int FTH, int COLOUR, bool ENERGY>
__device__ __forceinline__ int generic_colour(LdsT<FTH>& L, const SweepFusedArgs& a, const uint16_t* items,
                                                    int n_items, int ty0, int tx0, uint32_t r_global, int tid)
{
    constexpr int OC = COLOUR ^ 1;
    constexpr int CW = Tile<FTH>::CW;
    const uint32_t w3 = ctr_word3(a.scene, TAG_SWEEP, (uint32_t)COLOUR);
    const uint32_t pm_base = (uint32_t)(tx0 / 4) - 1u;
    int e_sum = 0;
    for (int it = tid; it < n_items; it += Tile<FTH>::FS_NT) {
        const unsigned code = items[it];
        const int yl = (int)(code >> 8), pl = (int)((code >> 2) & 63u), sm = (int)(code & 3u);
        const int gy = ty0 - 2 + yl;
        const int delta = (gy + COLOUR) & 1;
        const int Ja = 2 * pl + 2;
        const U4 w = philox_x3((uint32_t)gy * (uint32_t)a.Mw + pm_base + (uint32_t)pl, a.sweep, r_global, w3, a.key0,
                               a.key1);
        const int row_b = L.brow[yl];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!((sm >> h) & 1)) continue;
            const int J = Ja + h;
            const int i_own = (COLOUR * Tile<FTH>::RH + yl) * CW + J;
            const int i_mid = (OC * Tile<FTH>::RH + yl) * CW + J;
            const int i_u = i_mid - CW, i_d = i_mid + CW, i_l = i_mid - 1 + delta, i_r = i_mid + delta;
            const float2* const cs = &L.cs[0][0][0];
            const int xl = 4 * (pl - 1) + delta + 2 * h + 2;     // region column
            const int bidx = row_b + L.bcol[xl];
            const TBand tb = a.Tb[bidx];
            e_sum += site_update<FTH, ENERGY>(L, a, cs[i_own], cs[i_u], cs[i_l], cs[i_r], cs[i_d], h ? w.z : w.x,
                                              h ? w.w : w.y, tb, i_own, i_u, i_l, i_r, i_d);
        }
    }
    return e_sum;
}

// Energy / J of all bonds of a colour-1 site at (yl, J) from the LDS values.
template <int FTH>
__device__ __forceinline__ float site_energy1(const LdsT<FTH>& L, int yl, int J, int delta)
{
    const float2 o = L.cs[1][yl][J];
    const float2 u = L.cs[0][yl - 1][J], d = L.cs[0][yl + 1][J];
    const float2 l = L.cs[0][yl][J - 1 + delta], rt = L.cs[0][yl][J + delta];
    const float Cx = ((u.x + l.x) + rt.x) + d.x;
    const float Sy = ((u.y + l.y) + rt.y) + d.y;
    return -fmaf(o.x, Cx, o.y * Sy);
}

// One sweep of tile `tile` (row-major in a.ntx x a.nty tiles) for realizations
// [chunk * a.rchunk, min(R, (chunk + 1) * a.rchunk)).  Every thread of the workgroup must call it; LDS is free
// again when it returns.
template <int FTH>
__device__ __forceinline__ void sweep_tile(LdsT<FTH>& L, const SweepFusedArgs& a, int tile, int chunk)
{
    using C = Tile<FTH>;
    constexpr int FT_W = C::FT_W, FT_H = C::FT_H, FS_NT = C::FS_NT, RH = C::RH, RW = C::RW, CW = C::CW;
    constexpr int NPR = C::NPR, MAX_RED = C::MAX_RED, MAX_BLK = C::MAX_BLK, MAX_EOBS = C::MAX_EOBS;
    constexpr int MAIN_K = C::MAIN_K, CPT = C::CPT;
    // opaque thread index: nothing derived from it is hoisted out of a caller's item loop (register pressure)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int tx0 = (tile % a.ntx) * FT_W, ty0 = (tile / a.ntx) * FT_H;
    const int W = a.W, H = a.H;
    const int r_begin = chunk * a.rchunk;
    const int r_end = r_begin + a.rchunk < a.R ? r_begin + a.rchunk : a.R;

    // ---- setup 1: zero the cell arrays (outside cells stay (t = -0, cs = 0)), temperature-block tables ----
    {
        float* z = &L.cs[0][0][0].x;
        for (int i = tid; i < 2 * RH * CW * 2; i += FS_NT) z[i] = 0.0f;
        float* zt = &L.t[0][0][0];
        for (int i = tid; i < 2 * RH * CW; i += FS_NT) zt[i] = -0.0f;
    }
    const int gy_lo = ty0 - 2 > 0 ? ty0 - 2 : 0, gy_hi = ty0 + FT_H + 1 < H - 1 ? ty0 + FT_H + 1 : H - 1;
    const int gx_lo = tx0 - 2 > 0 ? tx0 - 2 : 0, gx_hi = tx0 + FT_W + 1 < W - 1 ? tx0 + FT_W + 1 : W - 1;
    const int by0 = gy_lo / a.lb_h, bx0 = gx_lo / a.lb_w;
    const int nby_l = gy_hi / a.lb_h - by0 + 1, nbx_l = gx_hi / a.lb_w - bx0 + 1;
    const bool use_table = nby_l * nbx_l <= C::TP_CAP;
    // fast lists: table temperatures, block columns made of whole pairs, counters within 24-bit products
    const bool fast = use_table && a.lb_w % 4 == 0 && a.Mw < (1 << 23);
    if (tid < RH) {
        const int gy = ty0 - 2 + tid;
        int v = 0;
        if (gy >= 0 && gy < H) v = fast ? (gy / a.lb_h - by0) * nbx_l : (gy / a.lb_h) * a.nbx;
        L.brow[tid] = v;
    } else if (tid >= 64 && tid < 64 + RW) {
        const int gx = tx0 - 2 + (tid - 64);
        int v = 0;
        if (gx >= 0 && gx < W) v = fast ? gx / a.lb_w - bx0 : gx / a.lb_w;
        L.bcol[tid - 64] = v;
    } else if (fast && tid >= 192 && tid < 192 + C::TP_CAP) {
        const int i = tid - 192;
        if (i < nby_l * nbx_l) L.tp[i] = a.Tb[(int64_t)(by0 + i / nbx_l) * a.nbx + bx0 + i % nbx_l];
    }
    __syncthreads();

    // ---- setup 2: sample cells (from any realization: samples are the same in all), gap bits of my cells ----
    const float* __restrict__ src0 = a.src + (int64_t)r_begin * a.HW;
    const int lane64 = tid & 63, row0 = tid >> 6;
    const int W4 = 4 * W;
    // my middle-column cells: region (row0 + 4k, 2 + lane64) = grid (ty0 - 2 + row0 + 4k, tx0 + lane64)
    const int gx_m = tx0 + lane64;
    const int off_m = (ty0 - 2 + row0) * W + gx_m;      // offsets within one realization (H W < 2^31)
    const int g_m = (ty0 + tx0 + row0 + lane64) & 1;
    const int J_m = cell_J(2 + lane64);
    // my side cell (threads < 4 RH): region (tid >> 2, {0, 1, 66, 67}[tid & 3])
    const int yl_s = tid >> 2;
    const int xl_s = (tid & 3) < 2 ? (tid & 3) : RW - 4 + (tid & 3);
    const int gy_s = ty0 - 2 + yl_s, gx_s = tx0 - 2 + xl_s;
    const int off_s = gy_s * W + gx_s;
    const int g_s = (ty0 + tx0 + yl_s + xl_s) & 1;
    const int J_s = cell_J(xl_s);
    const bool side_in = tid < 4 * RH && gy_s >= 0 && gy_s < H && gx_s >= 0 && gx_s < W;
    uint32_t gapbits = 0;
#pragma unroll
    for (int k = 0; k < MAIN_K; ++k) {
        const int gy = ty0 - 2 + row0 + 4 * k;
        if (gy >= 0 && gy < H && gx_m < W) {
            const int n = off_m + k * W4;
            if (a.mask[n]) {
                const float v = src0[n];
                const float ang = a.q * v;
                L.t[g_m][row0 + 4 * k][J_m] = -v;
                L.cs[g_m][row0 + 4 * k][J_m] = make_float2(cos_rev(ang), sin_rev(ang));
            } else {
                gapbits |= 1u << k;
            }
        }
    }
    if (side_in) {
        if (a.mask[off_s]) {
            const float v = src0[off_s];
            const float ang = a.q * v;
            L.t[g_s][yl_s][J_s] = -v;
            L.cs[g_s][yl_s][J_s] = make_float2(cos_rev(ang), sin_rev(ang));
        } else {
            gapbits |= 1u << MAIN_K;
        }
    }
    // first realization's gap cells into registers, and mark the gap cells (positive) for the lists below
    float pre[CPT];
#pragma unroll
    for (int k = 0; k < MAIN_K; ++k) {
        pre[k] = 0.0f;
        if ((gapbits >> k) & 1u) {
            pre[k] = src0[off_m + k * W4];
            L.t[g_m][row0 + 4 * k][J_m] = 0.5f;
        }
    }
    pre[MAIN_K] = 0.0f;
    if ((gapbits >> MAIN_K) & 1u) {
        pre[MAIN_K] = src0[off_s];
        L.t[g_s][yl_s][J_s] = 0.5f;
    }
    __syncthreads();

    // ---- setup 3: compacted lists (deterministic order); colour 0 in items[0 .. MAX_RED), colour 1 after ----
    // Fast codes: bits 0..10 the LDS index of the lowest cell read (pair: float4 index; single site: float2 index),
    // bits 11..15 the temperature-table index.  Generic codes: row << 8 | pair << 2 | site mask.
    uint16_t* const list0 = L.items;
    uint16_t* const list1 = L.items + MAX_RED;
    int nf0 = 0, nh0 = 0, nf1 = 0, nh1 = 0;
    for (int base = 0; base < MAX_RED; base += FS_NT) {
        const int i = base + tid;
        unsigned sm = 0;
        int yl = 0, pl = 0, delta = 0;
        if (i < MAX_RED) {
            yl = 1 + i / NPR;
            pl = i % NPR;
            delta = (ty0 - 2 + yl) & 1;           // colour 0
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int xrel = 4 * (pl - 1) + delta + 2 * h;
                if (xrel >= -1 && xrel <= FT_W && !is_fixed(L.t[0][yl][cell_J(xrel + 2)])) sm |= 1u << h;
            }
        }
        if (fast) {
            const int hfree = sm == 2u ? 1 : 0;
            const unsigned tix = sm ? (unsigned)(L.brow[yl] + L.bcol[4 * (pl - 1) + delta + 2 * hfree + 2]) : 0u;
            const unsigned a4 = (unsigned)(20 * yl + pl + 1);
            const int cat = sm == 3u ? 1 : (sm ? 2 : 0);
            const unsigned idx = cat == 1 ? a4 : 2u * a4 + (unsigned)hfree;
            compact2(cat, (uint16_t)(idx | tix << 11), list0, MAX_RED, nf0, nh0, L.wcnt);
        } else {
            nf0 = compact(sm != 0, (uint16_t)((yl << 8) | (pl << 2) | sm), list0, nf0, L.wcnt[0]);
        }
    }
    for (int base = 0; base < MAX_BLK; base += FS_NT) {
        const int i = base + tid;
        unsigned sm = 0;
        int yl = 0, pl = 0, delta = 0;
        if (i < MAX_BLK) {
            yl = 2 + i / (FT_W / 4);
            pl = 1 + i % (FT_W / 4);
            delta = (ty0 - 2 + yl + 1) & 1;       // colour 1
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int xrel = 4 * (pl - 1) + delta + 2 * h;
                if (!is_fixed(L.t[1][yl][cell_J(xrel + 2)])) sm |= 1u << h;
            }
        }
        if (fast) {
            const int hfree = sm == 2u ? 1 : 0;
            const unsigned tix = sm ? (unsigned)(L.brow[yl] + L.bcol[4 * (pl - 1) + delta + 2 * hfree + 2]) : 0u;
            const unsigned a4 = (unsigned)(20 * (yl - 1) + pl + 1);    // the cell above the pair's left site
            const int cat = sm == 3u ? 1 : (sm ? 2 : 0);
            const unsigned idx = cat == 1 ? a4 : 2u * a4 + (unsigned)hfree;
            compact2(cat, (uint16_t)(idx | tix << 11), list1, MAX_BLK, nf1, nh1, L.wcnt);
        } else {
            nf1 = compact(sm != 0, (uint16_t)((yl << 8) | (pl << 2) | sm), list1, nf1, L.wcnt[0]);
        }
    }
    // Random-stream counter of a pair: row * Mw + global pair index.  With q = LDS index / 20 (per pair) the row is
    // ty0 - 2 + q + colour and the pair index within the region is (LDS index) - 20 q - 1.
    const uint32_t pm_base = (uint32_t)(tx0 / 4) - 1u;
    const uint32_t ctr0 = (uint32_t)(ty0 - 2) * (uint32_t)a.Mw + pm_base - 1u;
    const uint32_t ctr1 = ctr0 + (uint32_t)a.Mw;
    // colour-1 sample sites of the tile: with a gap neighbour -> list; otherwise their energy is constant
    int ne = 0;
    long long e_const = 0;
    for (int base = 0; base < MAX_EOBS; base += FS_NT) {
        const int i = base + tid;
        bool f = false;
        uint16_t code = 0;
        const int yl = 2 + i / (FT_W / 2);
        const int gy = ty0 - 2 + yl;
        const int delta = (gy + 1) & 1;
        const int xrel = 2 * (i % (FT_W / 2)) + delta;
        const int J = cell_J(xrel + 2);
        if (i < MAX_EOBS && gy < H && tx0 + xrel < W && is_fixed(L.t[1][yl][J])) {
            const bool touches_gap = !is_fixed(L.t[0][yl - 1][J]) || !is_fixed(L.t[0][yl + 1][J]) ||
                                     !is_fixed(L.t[0][yl][J - 1 + delta]) || !is_fixed(L.t[0][yl][J + delta]);
            if (touches_gap) {
                f = true;
                code = (uint16_t)((yl << 8) | J);
            } else {
                e_const += to_fix(site_energy1<FTH>(L, yl, J, delta));
            }
        }
        ne = compact(f, code, L.eobs, ne, L.wcnt[0]);
    }
    // the workgroup's constant part, summed once (scalar registers)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e_const += __shfl_xor(e_const, off, 64);
    if ((tid & 63) == 0) L.red[tid >> 6] = e_const;
    __syncthreads();
    {
        const long long c = ((L.red[0] + L.red[1]) + L.red[2]) + L.red[3];
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(unsigned long long)c);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)c >> 32));
        e_const = (long long)(((unsigned long long)hi << 32) | lo);
    }
    __syncthreads();

    // ---- realizations ----
    for (int r = r_begin; r < r_end; ++r) {
        float* __restrict__ dst = a.dst + (int64_t)r * a.HW;
        // opaque per realization: the per-row offsets below are recomputed (one add each) instead of being kept as
        // 64-bit addresses across the loop; uniform base + unsigned 32-bit offset addressing
        int om = off_m, os = off_s, Wr = W;
        asm volatile("" : "+v"(om), "+v"(os), "+s"(Wr));
        const int W4r = 4 * Wr;
        // 1. gap cells from registers
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if ((gapbits >> k) & 1u) {
                const float v = pre[k];
                const float ang = a.q * v;
                const float2 cs = make_float2(cos_rev(ang), sin_rev(ang));
                if (k < MAIN_K) {
                    L.t[g_m][row0 + 4 * k][J_m] = v;
                    L.cs[g_m][row0 + 4 * k][J_m] = cs;
                } else {
                    L.t[g_s][yl_s][J_s] = v;
                    L.cs[g_s][yl_s][J_s] = cs;
                }
            }
        }
        __syncthreads();
        if (r + 1 < r_end) {
            const float* __restrict__ srcn = a.src + (int64_t)(r + 1) * a.HW;
#pragma unroll
            for (int k = 0; k < MAIN_K; ++k)
                if ((gapbits >> k) & 1u) pre[k] = srcn[(uint32_t)(om + k * W4r)];
            if ((gapbits >> MAIN_K) & 1u) pre[MAIN_K] = srcn[(uint32_t)os];
        }
        const uint32_t rg = a.real_offset + (uint32_t)r;
        // 2. colour 0 on tile + ring
        if (fast)
            fast_colour<FTH, 0, false>(L, a, list0, MAX_RED, nf0, nh0, ctr0, rg, tid);
        else
            generic_colour<FTH, 0, false>(L, a, list0, nf0, ty0, tx0, rg, tid);
        __syncthreads();
        // 3. colour 1 on the tile
        int e = 0;
        if (fast) {
            if (a.e_partial)
                e = fast_colour<FTH, 1, true>(L, a, list1, MAX_BLK, nf1, nh1, ctr1, rg, tid);
            else
                fast_colour<FTH, 1, false>(L, a, list1, MAX_BLK, nf1, nh1, ctr1, rg, tid);
        } else {
            if (a.e_partial)
                e = generic_colour<FTH, 1, true>(L, a, list1, nf1, ty0, tx0, rg, tid);
            else
                generic_colour<FTH, 1, false>(L, a, list1, nf1, ty0, tx0, rg, tid);
        }
        __syncthreads();
        // 4. sample sites bordering gaps, write-back
        if (a.e_partial) {
            for (int i = tid; i < ne; i += FS_NT) {
                const unsigned code = L.eobs[i];
                const int yl = (int)(code >> 8), J = (int)(code & 255u);
                e += to_fix(site_energy1<FTH>(L, yl, J, (ty0 - 2 + yl + 1) & 1));
            }
            long long v = e;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if ((tid & 63) == 0) L.red[tid >> 6] = v;
        }
        // the tile's cells are my middle-column cells shifted by two rows: rows row0 + 2 + 4k, k < FT_H / 4
#pragma unroll
        for (int k = 0; k < FT_H / 4; ++k) {
            const int yl = row0 + 2 + 4 * k;
            const float v = L.t[g_m][yl][J_m];
            if (is_fixed(v)) continue;                      // samples and cells outside the grid
            dst[(uint32_t)(om + (2 + 4 * k) * Wr)] = v;
        }
        __syncthreads();
        if (a.e_partial && tid == 0) {
            long long s = e_const;
#pragma unroll
            for (int i = 0; i < FS_NT / 64; ++i) s += L.red[i];
            a.e_partial[(int64_t)r * a.ntiles + tile] = s;
        }
    }
}

}  // namespace mpr
