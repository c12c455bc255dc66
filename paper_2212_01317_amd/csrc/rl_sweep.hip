// Realization-lane sweep: the single-checkerboard Metropolis sweep of Sec. 2.2.2 (block or site temperatures) for
// runs with many realizations, in a state layout with the realization innermost.
//
// Layout: S[g][n][l], n = y W + x, realization r = 64 g + l (R rounded up to a multiple of 64).  Lane l of a wave
// is realization 64 g + l, so the 64 lanes update the same site in 64 realizations, and the 256 bytes of a site are
// 256 bytes from those of the next site in the row: whether a site is a sample, its temperature, its random-stream
// counter and its neighbourhood are the same for the whole wave.  They are scalar data, decided by the scalar
// unit, and no lane idles on a sample site.
//
// A wave owns a band of B = kRlBand columns [x0, x0 + B) and a segment of rows [ys, ye) of one group of 64
// realizations, and streams the rows downwards with a window of four rows: (cos, sin) of each site of columns
// x0 - 2 .. x0 + B + 1 in registers, the angles in LDS.  Step y updates colour 0 of row y and then colour 1 of
// row y - 1, whose colour-0 neighbours (rows y - 2 .. y) are then current; a colour-0 update writes its cell at
// once, the colour-1 row is written after the next row has arrived.
// A row is requested two steps before it is updated, into the slot it then occupies; at its arrival its loaded angles
// go to a four-slot ring in LDS, from which its updates read their old angles, so nothing is read twice from memory
// and the angles do not hold vector registers for four steps.  Colour 0 is also updated one site outside the band
// (columns x0 - 1, x0 + B) and one row outside the segment (rows ys - 1, ye): these updates use the same
// counter-based random numbers and the same inputs as in the wave that owns the site, so they are bit-identical to
// it (and so are the duplicate writes), and the two columns beyond (x0 - 2, x0 + B + 1) are read only.  Sweep k
// reads `src` and writes `dst`; both hold the sample angles at the sample sites.  The rare exact decision, a function
// out of line (one copy of its code, which keeps the loop within the instruction cache), reads the neighbours'
// angles from memory (colour-1 neighbours from `src`, colour-0 neighbours, already updated, from `dst`).
//
// The update, the decision (FP32 filter, exact FP64 test inside its error band), the random numbers and the
// fixed-point energy of each colour-1 site are those of the fused sweep, so the chains, the energy series and the
// stopping sweep are identical.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "batched.hpp"
#include "metropolis.hpp"
#include "mpr_internal.hpp"
#include "philox_lane.hpp"

namespace mpr {

namespace {


__device__ __forceinline__ int fix24(float x) { return __float2int_rn(x * 16777216.0f); }

// The exact decision of one update, out of line (one copy of its code per kernel): the neighbours' angles from
// memory at the lane's realization (colour 0: the colour-1 neighbours from src; colour 1: the colour-0 neighbours,
// written earlier in this launch, from dst through the device-coherent path after all stores have completed), then
// the FP64 test.  An absent neighbour reads the cell itself (in the grid) and is excluded by `present`.
__device__ __noinline__ bool exact_site(const char* base, int64_t off, int64_t wrow, int j, int x, int y, int W, int H,
                                        uint32_t lane4, int col, float tp, float to, float ui, double two_pi_q,
                                        double J, float T)
{
    const bool pu = y > 0, pl = x > 0, pr = x + 1 < W, pd = y + 1 < H;
    const char* p = base + off + (int64_t)j * 256 + lane4;
    const int64_t du = pu ? -wrow : 0, dd = pd ? wrow : 0, dl = pl ? -256 : 0, dr = pr ? 256 : 0;
    float nu, nl, nr, nd;
    if (col == 0) {
        nu = *reinterpret_cast<const float*>(p + du);
        nl = *reinterpret_cast<const float*>(p + dl);
        nr = *reinterpret_cast<const float*>(p + dr);
        nd = *reinterpret_cast<const float*>(p + dd);
    } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        nu = __hip_atomic_load(reinterpret_cast<const float*>(p + du), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nl = __hip_atomic_load(reinterpret_cast<const float*>(p + dl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nr = __hip_atomic_load(reinterpret_cast<const float*>(p + dr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nd = __hip_atomic_load(reinterpret_cast<const float*>(p + dd), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned present = (pu ? 1u : 0u) | (pl ? 2u : 0u) | (pr ? 4u : 0u) | (pd ? 8u : 0u);
    return exact64(tp, to, nu, nl, nr, nd, present, two_pi_q, J, T, ui * 5.9604644775390625e-8f);
}

// How a window column finds its temperature column: TM_ALIGNED when the blocks are a multiple of the band wide
// (the owned columns share one temperature column, each ring column may have its own), TM_TWO when the blocks are
// at least kRlBand + 3 wide (the window spans at most two temperature columns: those below `jsplit` take `bca`, the
// others `bcb`), TM_ANY otherwise (one division per column).
enum { TM_ANY = 0, TM_ALIGNED = 1, TM_TWO = 2 };

// DIR: directional coupling (a temperature per bond direction, table TBandDir); else one temperature (TBand).
template <int KB, int TM, bool ENERGY, bool DIR>
struct RlWave {
    static constexpr int kB = KB;          // columns owned by the wave
    static constexpr int kWC = KB + 4;     // window columns x0 - 2 .. x0 + KB + 1
    static constexpr uint32_t kAll = (1u << kWC) - 1u;
    using TB = typename std::conditional<DIR, TBandDir, TBand>::type;
    RlArgs a;
    const uint2* __restrict__ cells;   // [(H + 4) * nbands]: row y + 2 -> {gap bits, sample bits} of the window
    const TB* __restrict__ tb;
    const char* src;                   // this wave's group of realizations in the two state buffers
    char* dst;
    int band, x0, ys, ye, lane;
    uint32_t real;                     // global realization index of this lane
    PhiloxLane pl;                     // the lane's constant parts of the first two Philox rounds
    RoundKeys rk;                      // the round keys of rounds 2 .. 9
    uint32_t lane4;                    // byte offset of this lane inside a site's 64 realizations
    int64_t offy;                      // byte offset of (row y of the current step, window column 0) in the group
    int64_t wrow;                      // bytes per grid row: W * 256
    // window of (cos, sin), slot = row & 3
    float c[4][kWC], s[4][kWC];
    uint32_t gap[4], smp[4];           // per slot: gap / sample bits of the window columns
    float ang[4][kWC];                 // per slot: the angles of the row as loaded (requested two steps ahead),
                                       // until the row arrives
    float* sang;                       // LDS [4 slots][kWC][64]: the old angles of the arrived rows, by slot
    uint32_t pgap, psmp;
    uint2 nbits;                       // gap / sample bits of the next row to be requested, loaded one request ahead
    int brow, brem;                    // temperature row of the step's row y, and y - brow tb_h
    const TB* trow0;                   // temperature rows of y and y - 1 (clamped into the grid)
    const TB* trow1;
    const TB* tA0;                     // TM_TWO: the entries bca and bcb of the rows of y and y - 1
    const TB* tB0;
    const TB* tA1;
    const TB* tB1;
    int bc, bcl, bcr;                  // TM_ALIGNED: temperature columns of the owned columns and of the two ring columns
    int bca, bcb, jsplit;              // TM_TWO: the two temperature columns and the first window column of bcb
    long long e_acc;
    // Colour-1 results are written one step late, after the next row has arrived: no other wave reads a colour-1
    // cell in this sweep (this wave's exact tests read colour-1 neighbours from src), and the arrival then does not
    // wait for stores that were issued just before it.  (Not with DIR, whose larger update leaves no registers.)
    float pend[kWC];                   // new angles of the last colour-1 row, by window column
    uint32_t pend_gap;                 // its gap bits (0: nothing pending)
    int64_t pend_off;                  // its byte offset

    // the lane's element of window column j of the row at byte offset off (wave-uniform base + lane offset + an
    // immediate j * 256)
    __device__ __forceinline__ float ld(const char* b, int64_t off, int j) const
    {
        return *reinterpret_cast<const float*>(b + off + j * 256 + lane4);
    }
    __device__ __forceinline__ void st(int64_t off, int j, float v) const
    {
        *reinterpret_cast<float*>(dst + off + j * 256 + lane4) = v;
    }
    // the same load through the device-coherent path (values this wave stored earlier in the launch)
    __device__ __forceinline__ float ld_coherent(const char* b, int64_t off, int j) const
    {
        return __hip_atomic_load(reinterpret_cast<const float*>(b + off + j * 256 + lane4), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    }

    // temperature column of window column j (clamped into the grid), by the reciprocal tb_w_inv = ceil(2^32 / tb_w)
    __device__ __forceinline__ int bcol(int j) const
    {
        int x = x0 - 2 + j;
        x = x < 0 ? 0 : (x >= a.W ? a.W - 1 : x);
        return a.tb_w == 1 ? x : (int)__umulhi((uint32_t)x, a.tb_w_inv);
    }

    // (through the constant address space: a scalar load whatever the compiler can prove about aliasing)
    __device__ __forceinline__ uint2 row_bits(int y) const
    {
        using CU = const __attribute__((address_space(4))) uint32_t;
        const uint64_t ad = (uint64_t)(cells + ((int64_t)(y + 2) * a.nbands + band));
        const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)ad);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(ad >> 32));
        const CU* p = (const CU*)(lo | hi << 32);
        return make_uint2(p[0], p[1]);
    }

    // Requests the angles of the cells of row y that lie inside the grid (gap and sample cells alike: both state
    // buffers hold the sample angles) into slot S.
    template <int S>
    __device__ __forceinline__ void request(int y, int64_t off)
    {
        // rows are requested in order: the bits of row y were loaded by the previous request; load those of row
        // y + 1 now (clamped to the last row the table holds, H + 1; rows beyond it are never requested)
        const uint2 b = nbits;
        nbits = row_bits(y + 1 <= a.H + 1 ? y + 1 : a.H + 1);
        pgap = b.x;
        psmp = b.y;
        const uint32_t in = pgap | psmp;
        if (in == kAll) {
#pragma unroll
            for (int j = 0; j < kWC; ++j) ang[S][j] = ld(src, off, j);
        } else {
            // a cell outside the grid is not loaded: its slot entry is given no value (it is never read), which
            // ends the live range of the entry it replaces
#pragma unroll
            for (int j = 0; j < kWC; ++j)
                ang[S][j] = ((in >> j) & 1u) ? ld(src, off, j) : __builtin_nondeterministic_value(0.0f);
        }
    }

    // Row y enters slot S: (cos, sin) of the requested angles; cells outside the grid get (0, 0).  The (cos, sin)
    // of every window column are computed from whatever the slot holds and then cleared outside the grid, so that
    // the common case writes the slot once.
    __device__ __forceinline__ float& old_angle(int S, int j) const { return sang[(S * kWC + j) * 64 + lane4 / 4]; }

    template <int S>
    __device__ __forceinline__ void arrive()
    {
        gap[S] = pgap;
        smp[S] = psmp;
#pragma unroll
        for (int j = 0; j < kWC; ++j) {
            const float t = a.q * ang[S][j];
            c[S][j] = cos_rev(t);
            s[S][j] = sin_rev(t);
            if (j >= 1 && j < kWC - 1) old_angle(S, j) = ang[S][j];
            ang[S][j] = __builtin_nondeterministic_value(0.0f);
        }
        const uint32_t in = pgap | psmp;
        if (in != kAll) {
#pragma unroll
            for (int j = 0; j < kWC; ++j)
                if (!((in >> j) & 1u)) {
                    c[S][j] = 0.0f;
                    s[S][j] = 0.0f;
                }
        }
    }

    // Metropolis update of the gap cell at window column j of row y (slot SO; neighbours in slots SU above and SD
    // below), old angle `to`; writes the cell's angle after the update to dst.  COL = colour of the cell: colour-0
    // neighbours are read back from dst (this wave wrote them), colour-1 neighbours from src, on the exact path.
    // Returns the fixed-point energy / J of the site's bonds after the update.
    template <int COL, int SO, int SU, int SD>
    __device__ __forceinline__ int update(const TB& T, int y, int64_t off, int j, float to, uint32_t wp,
                                          uint32_t wa)
    {
        const float Cx = ((c[SU][j] + c[SO][j - 1]) + c[SO][j + 1]) + c[SD][j];
        const float Sy = ((s[SU][j] + s[SO][j - 1]) + s[SO][j + 1]) + s[SD][j];
        const float tp = u24(wp);
        const float ui = (float)(wa >> 8);
        const float ang = a.q * tp;
        const float cp = cos_rev(ang), sp = sin_rev(ang);
        const float co = c[SO][j], so = s[SO][j];
        if constexpr (DIR) return update_directional<COL, SO, SU, SD>(T, y, off, j, to, tp, ui, cp, sp, co, so, Cx, Sy);
        else {
        const float X = fmaf(cp - co, Cx, (sp - so) * Sy);
        // The FP32 filter with a wave-uniform temperature as a signed margin r and a tolerance: accept iff r < 0,
        // exact FP64 test iff |r| <= tol.  T > 0: r = ui - w24 (its sign is that of the exact difference, and it is
        // 0 only when ui = w24) within the error band of w24; T = 0: r = dE within delta (dE < 0 and dE <= 0 differ
        // only at dE = 0, which lies inside the band).
        // both forms, then a select on T > 0 (a scalar integer test on the bits of T: the table holds T > 0 or +0;
        // for T = 0, kappa = 0 and the first form is finite and unused)
        const float w24 = exp2_fast(fminf(fmaf(X, T.kappa, 24.0f), 25.0f));
        const bool tpos = __float_as_int(T.T) > 0;
        const float r = tpos ? ui - w24 : -a.J * X;
        const float tol = tpos ? fmaf(w24, fmaf(fabsf(X), T.kb, T.band), 0.015625f) : a.delta_e;
        return decide<COL, SO>(r, tol, T, y, off, j, to, tp, ui, cp, sp, Cx, Sy);
        }
    }

    // The directional update: X_h from the left and right neighbours, X_v from the up and down neighbours,
    // y24 = fma(X_h, kx, fma(X_v, ky, 24)); the energy term is the unweighted bond energy, as for one temperature.
    template <int COL, int SO, int SU, int SD>
    __device__ __forceinline__ int update_directional(const TB& T, int y, int64_t off, int j, float to, float tp,
                                                      float ui, float cp, float sp, float co, float so, float Cx,
                                                      float Sy)
    {
        const float Ch = c[SO][j - 1] + c[SO][j + 1], Sh = s[SO][j - 1] + s[SO][j + 1];
        const float Cv = c[SU][j] + c[SD][j], Sv = s[SU][j] + s[SD][j];
        const float Xh = fmaf(cp - co, Ch, (sp - so) * Sh);
        const float Xv = fmaf(cp - co, Cv, (sp - so) * Sv);
        const float w24 = exp2_fast(fminf(fmaf(Xh, T.kx, fmaf(Xv, T.ky, 24.0f)), 25.0f));
        const float tol = fmaf(w24, fmaf(fabsf(Xh), T.kbx, fmaf(fabsf(Xv), T.kby, T.band)), 0.015625f);
        return decide<COL, SO>(ui - w24, tol, T, y, off, j, to, tp, ui, cp, sp, Cx, Sy);
    }

    // Completes the update of window column j of row y (slot SO) from the filter's margin r (accept iff r < 0)
    // and tolerance: where a lane has |r| <= tol, the whole wave reads the neighbours' angles and runs the exact
    // test, and those lanes take its decision (r = -1 or 1).  Then the window cell, the stored angle and the
    // fixed-point energy of the site's bonds.
    template <int COL, int SO>
    __device__ __forceinline__ int decide(float r, float tol, const TB& T, int y, int64_t off, int j, float to,
                                          float tp, float ui, float cp, float sp, float Cx, float Sy)
    {
        const bool need = fabsf(r) <= tol;
        if (__builtin_amdgcn_ballot_w64(need) != 0) {
            const bool ex = exact_at<COL>(T, y, off, j, tp, to, ui);
            r = need ? (ex ? -1.0f : 1.0f) : r;
        }
        const bool acc = r < 0.0f;
        const float cf = acc ? cp : c[SO][j], sf = acc ? sp : s[SO][j];
        c[SO][j] = cf;
        s[SO][j] = sf;
        if (COL == 1 && !DIR) pend[j] = acc ? tp : to;
        else st(off, j, acc ? tp : to);
        return ENERGY ? fix24(-fmaf(cf, Cx, sf * Sy)) : 0;
    }

    // The exact decision of the update of window column j of row y: the neighbours' angles from memory (colour-0
    // cells: colour-1 neighbours from src; colour-1 cells: colour-0 neighbours, written earlier in this launch,
    // from dst through the device-coherent path), then the FP64 test.  An absent neighbour reads the cell itself
    // (in the grid) and is excluded by `pres`.
    template <int COL>
    __device__ __forceinline__ bool exact_at(const TB& T, int y, int64_t off, int j, float tp, float to,
                                             float ui) const
    {
        if constexpr (!DIR) {
            int xb = x0;
            asm volatile("" : "+s"(xb));
            return exact_site(COL == 0 ? src : static_cast<const char*>(dst), off, wrow, j, xb - 2 + j, y, a.W, a.H,
                              lane4, COL, tp, to, ui, a.two_pi_q, a.Jd, T.T);
        } else {
            return exact_dir<COL>(T, y, off, j, tp, to, ui);
        }
    }
    template <int COL>
    __device__ __forceinline__ bool exact_dir(const TB& T, int y, int64_t off, int j, float tp, float to,
                                              float ui) const
    {
        // the band origin through an opaque copy: the per-column offsets below are then computed here, on this
        // rare path, instead of being kept for every window column for the whole launch
        int xb = x0;
        asm volatile("" : "+s"(xb));
        const int x = xb - 2 + j;
        const bool pu = y > 0, pl = x > 0, pr = x + 1 < a.W, pd = y + 1 < a.H;
        const int64_t ou = pu ? off - wrow : off, od = pd ? off + wrow : off;
        const int jl = pl ? j - 1 : j, jr = pr ? j + 1 : j;
        float nu, nl, nr, nd;
        if (COL == 0) {
            nu = ld(src, ou, j);
            nl = ld(src, off, jl);
            nr = ld(src, off, jr);
            nd = ld(src, od, j);
        } else {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            nu = ld_coherent(dst, ou, j);
            nl = ld_coherent(dst, off, jl);
            nr = ld_coherent(dst, off, jr);
            nd = ld_coherent(dst, od, j);
        }
        const unsigned pres = (pu ? 1u : 0u) | (pl ? 2u : 0u) | (pr ? 4u : 0u) | (pd ? 8u : 0u);
        const float u = ui * 5.9604644775390625e-8f;
        return exact64_directional(tp, to, nu, nl, nr, nd, pres, a.two_pi_q, a.Jd, T.Tx, T.Ty, u);
    }

    // The temperature entry of window column j in the row trow.  The table is read-only for the whole launch and the
    // address is wave-uniform: it is read through the constant address space, which makes it a scalar load.
    // ROW: 0 for row y (colour 0), 1 for row y - 1 (colour 1), the rows whose TM_TWO entries are tA0/tB0 and tA1/tB1
    template <int ROW>
    __device__ __forceinline__ TB tband(const TB* trow, int j) const
    {
        using CU = const __attribute__((address_space(4))) uint32_t;
        const int k = TM == TM_ALIGNED ? (j == 1 ? bcl : (j == kWC - 2 ? bcr : bc)) : (TM == TM_TWO ? 0 : bcol(j));
        const TB* e = TM == TM_TWO ? (j < jsplit ? (ROW == 0 ? tA0 : tA1) : (ROW == 0 ? tB0 : tB1)) : trow + k;
        const uint64_t ad = (uint64_t)e;
        const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)ad);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(ad >> 32));
        const CU* p = (const CU*)(lo | hi << 32);
        uint32_t w[sizeof(TB) / 4];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(TB) / 4); ++i) w[i] = p[i];
        TB t;
        __builtin_memcpy(&t, w, sizeof(TB));
        return t;
    }

    // Colour COL of the row in slot SO (grid row y): the pairs of groups m0 + MLO .. m0 + MHI, sites restricted to
    // window columns [JLO, JHI).  PAR = (y + COL) & 1, the column offset of the colour inside a group of four.
    template <int COL, int PAR, int SO, int SU, int SD, int MLO, int MHI, int JLO, int JHI>
    __device__ __forceinline__ int colour(const TB* trow, int y, int64_t off)
    {
        const uint32_t w3k1 = ctr_word3(a.scene, TAG_SWEEP, (uint32_t)COL) ^ a.key1;
        const uint32_t base = (uint32_t)y * (uint32_t)a.Mw + (uint32_t)(x0 / 4);
        int e = 0;
#pragma unroll
        for (int m = MLO; m <= MHI; ++m) {
            const int j0 = 4 * m + 2 + PAR, j1 = j0 + 2;
            const bool in0 = j0 >= JLO && j0 < JHI, in1 = j1 >= JLO && j1 < JHI;
            const int k0 = in0 ? j0 : JLO, k1 = in1 ? j1 : JLO;
            const bool g0 = in0 && ((gap[SO] >> k0) & 1u);
            const bool g1 = in1 && ((gap[SO] >> k1) & 1u);
            if (!(g0 || g1)) continue;
            const TB T0 = tband<COL>(trow, k0), T1 = tband<COL>(trow, k1);
            const float to0 = old_angle(SO, k0), to1 = old_angle(SO, k1);
            const U4 w = philox_site(base + (uint32_t)m, w3k1, pl, rk);
            if (g0) e += update<COL, SO, SU, SD>(T0, y, off, k0, to0, w.x, w.y);
            if (g1) e += update<COL, SO, SU, SD>(T1, y, off, k1, to1, w.z, w.w);
        }
        return e;
    }

    // Energy / J (fixed point) of the bonds of the colour-1 sample cells of the row in slot SO among the owned
    // columns (the gap cells' energies come from their updates).
    template <int PAR, int SO, int SU, int SD>
    __device__ __forceinline__ int sample_energy()
    {
        int e = 0;
#pragma unroll
        for (int k = 0; k < kB / 2; ++k) {
            const int j = 2 + 2 * k + PAR;
            if (!((smp[SO] >> j) & 1u)) continue;
            const float Cx = ((c[SU][j] + c[SO][j - 1]) + c[SO][j + 1]) + c[SD][j];
            const float Sy = ((s[SU][j] + s[SO][j - 1]) + s[SO][j + 1]) + s[SD][j];
            e += fix24(-fmaf(c[SO][j], Cx, s[SO][j] * Sy));
        }
        return e;
    }

    // One step (P = y & 3): row y + 1 arrives, row y + 2 is requested, colour 0 of row y, colour 1 of row y - 1.
    // The old angles of the step's updates are those its rows were loaded with.
    template <int P>
    __device__ __forceinline__ void step(int y)
    {
        constexpr int S0 = P, SU = (P + 3) & 3, SD = (P + 1) & 3, S2 = (P + 2) & 3;
        // temperature rows: trow1 <- row y - 1, trow0 <- row y
        trow1 = trow0;
        if (++brem == a.tb_h) {
            brem = 0;
            ++brow;
        }
        trow0 = tb + (int64_t)(brow < 0 ? 0 : (brow >= a.nby_t ? a.nby_t - 1 : brow)) * a.nbx_t;
        if (TM == TM_TWO) {
            tA1 = tA0;
            tB1 = tB0;
            tA0 = trow0 + bca;
            tB0 = trow0 + bcb;
        }
        // keeps the per-column choice of TM_TWO from being hoisted out of the row loop as a table of pointers
        if (TM == TM_TWO) asm volatile("" : "+s"(jsplit));
        offy += wrow;
        // row parity: y & 1 = P & 1, so colour 0 of row y and colour 1 of row y - 1 have column offset P & 1.
        const int y1 = y - 1;
        const bool do0 = y >= 0 && y < a.H, do1 = y1 >= ys && y1 < ye;
        arrive<SD>();
        flush<(P + 1) & 1>();
        if (y + 2 <= ye + 1) request<S2>(y + 2, offy + 2 * wrow);
        else pgap = psmp = 0u;
        if (do0) colour<0, P & 1, S0, SU, SD, -1, kB / 4, 1, kWC - 1>(trow0, y, offy);
        if (do1) {
            int e = colour<1, P & 1, SU, S2, S0, 0, kB / 4 - 1, 2, kWC - 2>(trow1, y1, offy - wrow);
            if (ENERGY) e += sample_energy<P & 1, SU, S2, S0>();
            e_acc += e;
            if (!DIR) {
                pend_gap = gap[SU];
                pend_off = offy - wrow;
            }
        }
    }

    // Writes the pending colour-1 row (column offset PAR: window columns 2 + PAR, 4 + PAR, ... 12 + PAR).
    template <int PAR>
    __device__ __forceinline__ void flush()
    {
        if (pend_gap != 0u) {
#pragma unroll
            for (int j = 2 + PAR; j < kWC - 2; j += 2)
                if ((pend_gap >> j) & 1u) st(pend_off, j, pend[j]);
        }
        pend_gap = 0u;
        // the pending angles are dead until the next colour-1 row writes them
#pragma unroll
        for (int j = 0; j < kWC; ++j) pend[j] = __builtin_nondeterministic_value(0.0f);
    }

    __device__ __forceinline__ void run()
    {
        e_acc = 0;
        pl = philox_lane(real, a.sweep, a.key0, a.key1);
        rk = round_keys(a.key0, a.key1);
        if (TM == TM_TWO) {
            bca = bcol(0);
            bcb = bcol(kWC - 1);
            jsplit = 0;
            if (bca != bcb)
                for (int j = 0; j < kWC; ++j) jsplit += bcol(j) == bca ? 1 : 0;
            jsplit = __builtin_amdgcn_readfirstlane(jsplit);
        }
        if (TM == TM_ALIGNED) {
            bc = x0 / a.tb_w;
            bcl = x0 % a.tb_w == 0 && bc > 0 ? bc - 1 : bc;
            bcr = (x0 + kB) % a.tb_w == 0 && bc + 1 < a.nbx_t ? bc + 1 : bc;
        }
        // the first step is y = ys - 1 (>= -1): start the temperature row one row above it
        brow = (ys - 2 + a.tb_h) / a.tb_h - 1;
        brem = (ys - 2 + a.tb_h) % a.tb_h;
        trow0 = tb;
        if (TM == TM_TWO) {
            tA0 = tb + bca;
            tB0 = tb + bcb;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < kWC; ++j) ang[i][j] = 0.0f;
        wrow = (int64_t)a.W * 256;
        offy = ((int64_t)(ys - 2) * a.W + (x0 - 2)) * 256;   // row ys - 2; the first step moves it to ys - 1
        // rows ys - 2 and ys - 1 into their slots (ys is a multiple of 4: slots 2 and 3), row ys requested
        nbits = row_bits(ys - 2);
        request<2>(ys - 2, offy);
        arrive<2>();
        request<3>(ys - 1, offy + wrow);
        arrive<3>();
        request<0>(ys, offy + 2 * wrow);
        pend_gap = 0u;
        for (int yb = ys - 1; yb <= ye; yb += 4) {
            step<3>(yb);
            if (yb + 1 > ye) break;
            step<0>(yb + 1);
            if (yb + 2 > ye) break;
            step<1>(yb + 2);
            if (yb + 3 > ye) break;
            step<2>(yb + 3);
        }
        // the colour-1 row of the last step (y = ye, column offset ye & 1)
        if (ye & 1) flush<1>();
        else flush<0>();
    }
};

// A band starts on a column that is a multiple of 4 (its Philox pairs are whole: pair index x0 / 4 + m), a segment on
// a row that is a multiple of 4 (window slot = row & 3, colour parity = slot parity).
static_assert(kRlBand % 4 == 0, "bands must start on a multiple of 4 columns");
static_assert(kRlSegRows % 4 == 0, "row segments must start on a multiple of 4 rows");

template <int TM, bool ENERGY, bool DIR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kRlWaves, kRlWaves))) void k_sweep_rl(
    RlArgs a, const uint2* __restrict__ cells, const void* __restrict__ tbv, const float* __restrict__ src,
    float* __restrict__ dst, long long* __restrict__ epart)
{
    // XCD-aware order: workgroup g runs on XCD g % 8; consecutive items (adjacent bands) go to the same XCD.
    const uint32_t N = a.n_items;
    const uint32_t g = blockIdx.x, xcd = g & 7u, k = g >> 3;
    const uint32_t per = N >> 3, rem = N & 7u;
    const uint32_t item = xcd < rem ? xcd * (per + 1u) + k : rem * (per + 1u) + (xcd - rem) * per + k;
    if (item >= N) return;
    const int64_t group = (int64_t)(item / ((uint32_t)a.nbands * (uint32_t)a.nseg)) * ((int64_t)a.H * a.W * 256);
    using TB = typename RlWave<kRlBand, TM, ENERGY, DIR>::TB;
    const TB* tb = static_cast<const TB*>(tbv);
    __shared__ float sang[4 * (kRlBand + 4) * 64];
    RlWave<kRlBand, TM, ENERGY, DIR> w{a, cells, tb, reinterpret_cast<const char*>(src) + group,
                                       reinterpret_cast<char*>(dst) + group};
    w.sang = sang;
    w.band = (int)(item % (uint32_t)a.nbands);
    const uint32_t rest = item / (uint32_t)a.nbands;
    const int seg = (int)(rest % (uint32_t)a.nseg);
    const int rg = (int)(rest / (uint32_t)a.nseg);
    w.lane = (int)(rg * 64 + threadIdx.x);
    w.lane4 = threadIdx.x * 4u;
    w.real = a.real_offset + (uint32_t)w.lane;
    w.x0 = w.band * kRlBand;
    w.ys = seg * a.seg_rows;
    w.ye = w.ys + a.seg_rows < a.H ? w.ys + a.seg_rows : a.H;
    w.run();
    if (ENERGY && w.lane < a.R) epart[(int64_t)w.lane * (a.nbands * a.nseg) + seg * a.nbands + w.band] = w.e_acc;
}

// The batched form on the lane sweep: one persistent launch per sweep in which every wave takes work items from the
// queue of its XCD (workgroup g runs on XCD g % 8 and takes the items of the XCD's eighth of the work list, in order,
// so that adjacent bands of a scene share that XCD's L2) until the queue is empty.  The work list numbers the items
// (group of realizations, band, segment, as in k_sweep_rl) of the scenes still running, largest scenes first;
// every scene sweeps with its own arguments (scene id, temperatures, buffers) and the batch's sweep index, so its
// chains are those of its single-scene run.  The energy partials are written for the scenes that equilibrate.
// The loop's own state (the XCD's item range, the sweep index) and what the energy store needs after an item (the
// scene, segment and band) are kept in LDS and read back where needed, so that they hold no scalar registers while
// the wave sweeps (the sweep itself needs all of them).
struct BatchLaneLoop {
    int64_t first, last;
    int k, sidx, seg, band;
};

__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32)) << 32) |
                     (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)x));
}

template <int TM, bool ENERGY>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kRlWaves, kRlWaves))) void k_batchl_sweep(
    const BatchLaneScene* __restrict__ scenes, const BatchRun* __restrict__ runs, const int* __restrict__ order,
    const int64_t* __restrict__ prefix, BatchLaneCtl* ctl, int n_scenes)
{
    __shared__ float sang[4 * (kRlBand + 4) * 64];
    __shared__ BatchLaneLoop L;
    volatile BatchLaneLoop& VL = L;
    if (threadIdx.x == 0) {
        const uint32_t xcd = blockIdx.x & 7u;
        VL.first = ctl->bound[xcd];
        VL.last = ctl->bound[xcd + 1];
        VL.k = ctl->k;
    }
    __syncthreads();
    for (;;) {
        unsigned long long v = 0ull;
        if (threadIdx.x == 0) v = atomicAdd(&ctl->queue[blockIdx.x & 7u], 1ull);
        // lane 0's ticket, for the whole wave (a scalar value)
        const int64_t item = uniform64(VL.first) + (int64_t)uniform64((int64_t)v);
        if (item >= uniform64(VL.last)) break;
        int lo = 0, hi = n_scenes;            // largest i with prefix[i] <= item
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int sidx = order[lo];
        // the scene's descriptor through the constant address space: scalar loads (the kernel's stores cannot reach
        // it), so its fields are scalar values
        BatchLaneScene d;
        {
            using CU = const __attribute__((address_space(4))) uint32_t;
            const uint64_t sad = (uint64_t)(scenes + sidx);
            const CU* p = (const CU*)((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)sad) |
                                      ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(sad >> 32))
                                       << 32));
            uint32_t wds[sizeof(BatchLaneScene) / 4];
#pragma unroll
            for (int i = 0; i < (int)(sizeof(BatchLaneScene) / 4); ++i) wds[i] = p[i];
            __builtin_memcpy(&d, wds, sizeof(BatchLaneScene));
        }
        RlArgs a = d.a;
        const int k = __builtin_amdgcn_readfirstlane(VL.k);
        a.sweep = (uint32_t)k;
        const uint32_t local = (uint32_t)(item - prefix[lo]);
        const uint32_t per_group = (uint32_t)a.nbands * (uint32_t)a.nseg;
        const uint32_t rg = local / per_group, rest = local % per_group;
        const int64_t group = (int64_t)rg * ((int64_t)a.H * a.W * 256);
        // sweep k reads buf[(k - 1) & 1] and writes buf[k & 1], chosen by a select: an index into the descriptor's
        // array would place the whole descriptor in scratch memory
        const bool odd = (k & 1) != 0;
        float* const src = odd ? d.buf[0] : d.buf[1];
        float* const dst = odd ? d.buf[1] : d.buf[0];
        RlWave<kRlBand, TM, ENERGY, false> w{a, d.cells, d.tb, reinterpret_cast<const char*>(src) + group,
                                             reinterpret_cast<char*>(dst) + group};
        w.sang = sang;
        w.band = (int)(rest % (uint32_t)a.nbands);
        const int seg = (int)(rest / (uint32_t)a.nbands);
        w.lane = (int)(rg * 64 + threadIdx.x);
        w.lane4 = threadIdx.x * 4u;
        w.real = a.real_offset + (uint32_t)w.lane;
        w.x0 = w.band * kRlBand;
        w.ys = seg * a.seg_rows;
        w.ye = w.ys + a.seg_rows < a.H ? w.ys + a.seg_rows : a.H;
        if (ENERGY && threadIdx.x == 0) {
            VL.sidx = sidx;
            VL.seg = seg;
            VL.band = w.band;
        }
        w.run();
        if (ENERGY) {
            const int s2 = __builtin_amdgcn_readfirstlane(VL.sidx);
            const BatchLaneScene& d2 = scenes[s2];
            if (runs[s2].phase == 0 && w.lane < d2.a.R)
                d2.epart[(int64_t)w.lane * d2.nparts + __builtin_amdgcn_readfirstlane(VL.seg) * d2.a.nbands +
                         __builtin_amdgcn_readfirstlane(VL.band)] = w.e_acc;
        }
        // the LDS ring and the loop state are reused by the next item: one wave's LDS operations complete in order
    }
}

// cells[(y + 2) * nbands + band] for y in [-2, H + 2): bit j of .x = (y, x0 - 2 + j) is a gap of the grid, of .y =
// it is a sample.
__global__ __launch_bounds__(256) void k_rl_cells(const uint8_t* __restrict__ mask, int H, int W, int nbands,
                                                   uint2* __restrict__ cells)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)(H + 4) * nbands;
    if (i >= total) return;
    const int y = (int)(i / nbands) - 2, band = (int)(i % nbands);
    uint32_t gb = 0u, sb = 0u;
    if (y >= 0 && y < H) {
        for (int j = 0; j < kRlBand + 4; ++j) {
            const int x = band * kRlBand - 2 + j;
            if (x < 0 || x >= W) continue;
            if (mask[(int64_t)y * W + x]) sb |= 1u << j;
            else gb |= 1u << j;
        }
    }
    cells[i] = make_uint2(gb, sb);
}

// [R][HW] -> [G][HW][64] (pad realizations get 0) into one or two buffers, 64 sites x 64 realizations per
// workgroup through LDS.
__global__ __launch_bounds__(256) void k_rl_to_lanes(const float* __restrict__ in, int64_t HW, int R,
                                                      float* __restrict__ out, float* __restrict__ out2)
{
    __shared__ float tile[64][65];
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int g = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int r = g * 64 + i;
        const int64_t n = n0 + tx;
        tile[i][tx] = (r < R && n < HW) ? in[(int64_t)r * HW + n] : 0.0f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t n = n0 + i;
        if (n < HW) {
            const int64_t o = ((int64_t)g * HW + n) * 64 + tx;
            out[o] = tile[tx][i];
            if (out2) out2[o] = tile[tx][i];
        }
    }
}

// [G][HW][64] -> [R][HW]
__global__ __launch_bounds__(256) void k_rl_from_lanes(const float* __restrict__ in, int64_t HW, int R,
                                                        float* __restrict__ out)
{
    __shared__ float tile[64][65];
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int g = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t n = n0 + i;
        tile[i][tx] = n < HW ? in[((int64_t)g * HW + n) * 64 + tx] : 0.0f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int r = g * 64 + i;
        const int64_t n = n0 + tx;
        if (r < R && n < HW) out[(int64_t)r * HW + n] = tile[tx][i];
    }
}

// acc[n] += sum over realizations (in order) of the gap angle; the first pass starts from 0.
// A workgroup sums 64 consecutive sites: per group of 64 realizations its waves read the gap sites' 256-byte
// realization rows (one coalesced load per site) into an LDS tile, and lane l of the first wave adds site n0 + l's
// realizations in order r = 0 .. R - 1 (the order of a loop over the realizations).  Sample sites are not read.
__global__ __launch_bounds__(256) void k_rl_accumulate(const float* __restrict__ S, const uint8_t* __restrict__ mask,
                                                        int64_t HW, int R, int first, double* __restrict__ acc)
{
    __shared__ float tile[64 * 65];                 // [site][realization], rows padded against bank conflicts
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int wv = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63u);
    const int64_t ns = n0 + l;
    const bool mine = wv == 0 && ns < HW;
    const bool gap = mine && !mask[ns];
    double v = gap && !first ? acc[ns] : 0.0;
    for (int g = 0; g * 64 < R; ++g) {
        for (int j = wv; j < 64; j += 4) {
            const int64_t n = n0 + j;
            if (n < HW && !mask[n]) tile[j * 65 + l] = S[((int64_t)g * HW + n) * 64 + l];
        }
        __syncthreads();
        if (gap) {
            const int m = R - g * 64 < 64 ? R - g * 64 : 64;
            for (int k = 0; k < m; ++k) v += (double)tile[l * 65 + k];
        }
        __syncthreads();
    }
    if (gap) acc[ns] = v;
    else if (mine && first) acc[ns] = 0.0;
}

}  // namespace

RlGeom rl_geometry(int64_t H, int64_t W, int R)
{
    RlGeom g;
    g.Rp = (R + 63) / 64 * 64;
    g.nbands = (int)((W + kRlBand - 1) / kRlBand);
    // row segments of kRlSegRows rows, halved (down to 32) while the grid has fewer than kRlTargetWaves waves:
    // each segment adds two ring rows of colour-0 updates
    // (segments start on rows that are multiples of 4: the first two rows of a segment's window go to slots 2 and 3,
    // and the colour of a step's rows follows from the slot; halved heights are rounded up to a multiple of 4)
    const int64_t groups = g.Rp / 64;
    g.seg_rows = kRlSegRows;
    while (g.seg_rows > 32 && (int64_t)g.nbands * ((H + g.seg_rows - 1) / g.seg_rows) * groups < kRlTargetWaves) {
        const int half = (g.seg_rows / 2 + 3) / 4 * 4;
        g.seg_rows = half > 32 ? half : 32;
    }
    g.nseg = (int)((H + g.seg_rows - 1) / g.seg_rows);
    g.n_items = (int64_t)g.nbands * g.nseg * groups;
    return g;
}

RlGeom rl_geometry_full(int64_t H, int64_t W, int R)
{
    RlGeom g;
    g.Rp = (R + 63) / 64 * 64;
    g.nbands = (int)((W + kRlBand - 1) / kRlBand);
    g.seg_rows = kRlSegRows;
    g.nseg = (int)((H + g.seg_rows - 1) / g.seg_rows);
    g.n_items = (int64_t)g.nbands * g.nseg * (g.Rp / 64);
    return g;
}

int rl_tm(int tb_w) { return tb_w % kRlBand == 0 ? TM_ALIGNED : (tb_w >= kRlBand + 3 ? TM_TWO : TM_ANY); }

hipError_t launch_rl_cells(const uint8_t* mask, int64_t H, int64_t W, uint2* cells, hipStream_t s)
{
    const RlGeom g = rl_geometry(H, W, 64);
    const int64_t total = (H + 4) * (int64_t)g.nbands;
    hipLaunchKernelGGL(k_rl_cells, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, mask, (int)H, (int)W,
                       g.nbands, cells);
    return hipGetLastError();
}

hipError_t launch_rl_to_lanes(const float* in, int64_t HW, int R, float* out, float* out2, hipStream_t s)
{
    const int Rp = (R + 63) / 64 * 64;
    hipLaunchKernelGGL(k_rl_to_lanes, dim3((unsigned)((HW + 63) / 64), (unsigned)(Rp / 64)), dim3(256), 0, s, in,
                       HW, R, out, out2);
    return hipGetLastError();
}

hipError_t launch_rl_from_lanes(const float* in, int64_t HW, int R, float* out, hipStream_t s)
{
    const int Rp = (R + 63) / 64 * 64;
    hipLaunchKernelGGL(k_rl_from_lanes, dim3((unsigned)((HW + 63) / 64), (unsigned)(Rp / 64)), dim3(256), 0, s, in,
                       HW, R, out);
    return hipGetLastError();
}

hipError_t launch_rl_accumulate(const float* S, const uint8_t* mask, int64_t HW, int R, int first, double* acc,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_rl_accumulate, dim3((unsigned)((HW + 63) / 64)), dim3(256), 0, s, S, mask, HW, R, first,
                       acc);
    return hipGetLastError();
}

hipError_t launch_sweep_rl(const RlArgs& a, const uint2* cells, const TBand* tb, const TBandDir* tbd, const float* src,
                           float* dst, long long* epart, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const int tm = rl_tm(a.tb_w);
    const dim3 grid((unsigned)a.n_items);
    const void* t = tbd ? static_cast<const void*>(tbd) : static_cast<const void*>(tb);
#define MPR_RL_LAUNCH(TMV, EN, DI) \
    hipLaunchKernelGGL((k_sweep_rl<TMV, EN, DI>), grid, dim3(64), 0, s, a, cells, t, src, dst, epart)
#define MPR_RL_LAUNCH_TM(EN, DI)                          \
    do {                                                  \
        if (tm == TM_ALIGNED) MPR_RL_LAUNCH(TM_ALIGNED, EN, DI); \
        else if (tm == TM_TWO) MPR_RL_LAUNCH(TM_TWO, EN, DI);     \
        else MPR_RL_LAUNCH(TM_ANY, EN, DI);                \
    } while (0)
    if (tbd) {
        if (epart) MPR_RL_LAUNCH_TM(true, true);
        else MPR_RL_LAUNCH_TM(false, true);
    } else {
        if (epart) MPR_RL_LAUNCH_TM(true, false);
        else MPR_RL_LAUNCH_TM(false, false);
    }
#undef MPR_RL_LAUNCH_TM
#undef MPR_RL_LAUNCH
    return hipGetLastError();
}

hipError_t launch_batchl_sweep(const BatchLaneDev& b, int grid, hipStream_t s)
{
    const bool en = b.cfg.energy != 0;
#define MPR_BL_LAUNCH(TMV, EN) \
    hipLaunchKernelGGL((k_batchl_sweep<TMV, EN>), dim3(grid), dim3(64), 0, s, b.scenes, b.runs, b.order, b.prefix, \
                       b.ctl, b.n)
    if (b.tm == TM_ALIGNED) {
        if (en) MPR_BL_LAUNCH(TM_ALIGNED, true);
        else MPR_BL_LAUNCH(TM_ALIGNED, false);
    } else if (b.tm == TM_TWO) {
        if (en) MPR_BL_LAUNCH(TM_TWO, true);
        else MPR_BL_LAUNCH(TM_TWO, false);
    } else {
        if (en) MPR_BL_LAUNCH(TM_ANY, true);
        else MPR_BL_LAUNCH(TM_ANY, false);
    }
#undef MPR_BL_LAUNCH
    return hipGetLastError();
}

}  // namespace mpr
