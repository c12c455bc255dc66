// The 3D lattice: the method on a D x H x W grid (the extension to three dimensions named in Sec. 4).  Reading: the
// same Hamiltonian (Eq. 1) over the six nearest neighbours of the simple cubic lattice with open boundaries, the
// checkerboard colours c = (x + y + z) mod 2, temperature blocks lb_d x lb_h x lb_w, and the plane's random stream
// with the row index z H + y in place of y and the colour (x + y + z) mod 2.
//
// The sweep keeps the realization-lane layout of the plane, S[g][n][64] with n = (z H + y) W + x, but is a pair of
// half-sweeps (one launch per colour): a colour-c half-sweep reads only colour-(1 - c) neighbours, which it does not
// change, so it runs in place, with no ring of redundant updates and no second buffer, and a rejected proposal
// writes nothing.  A wave owns kB3 columns [x0, x0 + kB3) of one row y and a segment of planes [zs, ze) of one group
// of 64 realizations, and streams along z with a window of four planes of its row in registers ((cos, sin) of
// columns x0 - 1 .. x0 + kB3), plus the rows y - 1 and y + 1 of the current plane at the updated columns; every row
// is requested two steps (rows y +- 1 one step) before it is used.  The colour-c columns of a plane alternate with
// z; for them to be known at compile time the launch takes the rows of one parity, so (y + c) mod 2 is a template
// argument: a sweep is four launches (colours 0, 1 times row parities).
//
// The update (independent uniform proposal, FP32 filter with its error band, exact FP64 decision inside the band,
// in the oracle's neighbour order back, up, left, right, down, front) and the fixed-point energy of the colour-1
// sites (every bond has one colour-1 end) follow the plane's kernels.
#include <hip/hip_runtime.h>

#include "metropolis.hpp"
#include "lattice3d.hpp"
#include "mpr_internal.hpp"
#include "philox_lane.hpp"

namespace mpr {

namespace {

constexpr int kW3 = kB3 + 2;        // window columns x0 - 1 .. x0 + kB3
constexpr int kH3 = kB3 / 2;        // updated columns of a plane (one colour)
static_assert(kB3 % 4 == 0, "a band starts on a multiple of 4 columns (whole Philox pairs)");
static_assert(kZSeg3 % 4 == 0, "plane segments start on a multiple of 4 planes (window slot = plane & 3)");

__device__ __forceinline__ int fix24(float x) { return __float2int_rn(x * 16777216.0f); }

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT, class T>
__device__ __forceinline__ T block_sum(T v, T* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

// The exact decision with up to six neighbours, evaluated as the definition writes it (the oracle's order: back,
// up, left, right, down, front; absent neighbours excluded by `present`).
__device__ __noinline__ bool exact64_6(float tp, float to, float nb, float nu, float nl, float nr, float nd, float nf,
                                       unsigned present, double two_pi_q, double J, float T, float u2)
{
    double acc = 0.0;
    const double dtp = (double)tp, dto = (double)to;
    if (present & 1u) acc += cos(two_pi_q * (dtp - (double)nb)) - cos(two_pi_q * (dto - (double)nb));
    if (present & 2u) acc += cos(two_pi_q * (dtp - (double)nu)) - cos(two_pi_q * (dto - (double)nu));
    if (present & 4u) acc += cos(two_pi_q * (dtp - (double)nl)) - cos(two_pi_q * (dto - (double)nl));
    if (present & 8u) acc += cos(two_pi_q * (dtp - (double)nr)) - cos(two_pi_q * (dto - (double)nr));
    if (present & 16u) acc += cos(two_pi_q * (dtp - (double)nd)) - cos(two_pi_q * (dto - (double)nd));
    if (present & 32u) acc += cos(two_pi_q * (dtp - (double)nf)) - cos(two_pi_q * (dto - (double)nf));
    const double dE = -J * acc;
    if ((double)T > 0.0) return (double)u2 < exp(-dE / (double)T);
    return dE <= 0.0;
}

// The exact decision of the update at byte offset `off` (the lane's element of site (x, y, z)): the site's old angle
// and its neighbours' angles from the state (the neighbours have colour 1 - c and do not change during this
// half-sweep; the site is written only after its decision); an absent neighbour reads the site itself and is
// excluded.
__device__ __noinline__ bool exact3_site(const char* base, int64_t off, int64_t wrow, int64_t wplane, int x, int y,
                                         int z, int D, int H, int W, float tp, float ui, double two_pi_q, double J,
                                         float T)
{
    const bool pb = z > 0, pu = y > 0, pl = x > 0, pr = x + 1 < W, pd = y + 1 < H, pf = z + 1 < D;
    const char* p = base + off;
    const float to = *reinterpret_cast<const float*>(p);     // the site's current angle (written only after this)
    const float nb = *reinterpret_cast<const float*>(p + (pb ? -wplane : 0));
    const float nu = *reinterpret_cast<const float*>(p + (pu ? -wrow : 0));
    const float nl = *reinterpret_cast<const float*>(p + (pl ? -256 : 0));
    const float nr = *reinterpret_cast<const float*>(p + (pr ? 256 : 0));
    const float nd = *reinterpret_cast<const float*>(p + (pd ? wrow : 0));
    const float nf = *reinterpret_cast<const float*>(p + (pf ? wplane : 0));
    const unsigned present = (pb ? 1u : 0u) | (pu ? 2u : 0u) | (pl ? 4u : 0u) | (pr ? 8u : 0u) | (pd ? 16u : 0u) |
                             (pf ? 32u : 0u);
    return exact64_6(tp, to, nb, nu, nl, nr, nd, nf, present, two_pi_q, J, T, ui * 5.9604644775390625e-8f);
}

// One wave of a workgroup of kNW3 waves that own the consecutive rows y0 .. y0 + kNW3 - 1 (wave w: row y0 + w) of
// one band, plane segment and group of realizations.  Rows y +- 1 of the current plane, at the columns the wave
// updates, are those rows' colour-(1 - c) cells, which this half-sweep does not change: each wave publishes its own
// row's colour-(1 - c) (cos, sin) of the next plane in LDS, and the first and last waves also load and publish the
// rows just outside the tile (y0 - 1, y0 + kNW3).  LDS exchange: xch[buffer = plane & 1][slot][k][lane] of
// (cos, sin), slot 0 = row y0 - 1, slot w + 1 = row y0 + w, slot kNW3 + 1 = row y0 + kNW3; k indexes the four
// columns x0 + 2k + PX of the row below or above, whose PX is the reader's.  A wave's column parity PX = (x + y + z
// + c) mod 2 relative to x0 depends on YC = (y + c) mod 2, a template argument of its methods; the two forms are
// dispatched per wave and per step.
// The launch arguments the plane loop reads (the others are used before the loop only), so that the loop keeps no
// more scalar registers than it needs: the exact decision's FP64 constants are recomputed from q and J there as
// the host computes them (2 pi q and J as doubles), the FP32 tolerance of T = 0 is kDeltaE3 J as on the host, the
// temperature block row is advanced plane by plane instead of divided, and the counter word of the sweep's colour
// is formed once.
struct Lat3Loop {
    int D, H, W, nbands, Mw, lb_w, lb_d;
    uint32_t lbw_inv, w3k1;
    float q, J, delta_e;
    int64_t bz_stride;                 // temperature blocks per block plane: nby nbx
};

template <bool ENERGY>
struct Wave3 {
    Lat3Loop a;
    const uint32_t* cells;             // [(D H) nbands] gap bits of the window columns of each row
    const TBand* tb;
    char* S;                           // this wave's group of realizations
    float2* xch;                       // LDS exchange of the workgroup
    int y, band, x0, zs, ze, wslot;
    uint32_t lane4, lane, real;
    PhiloxLane pl;
    RoundKeys rk;
    int64_t wrow, wplane;              // bytes per grid row and per plane
    int64_t orow;                      // byte offset of (plane 0, row y, window column 0) in the group
    int64_t hoff;                      // byte offset of the halo row from row y (0: this wave loads no halo row)
    int hslot;                         // its exchange slot
    uint32_t colmask;                  // window columns inside the grid
    int bzc, bzr;                      // temperature block plane of the current plane, and the plane's place in it
    int64_t byx;                       // (y / lb_h) nbx: the row's offset inside a block plane
    float c[4][kW3], s[4][kW3];        // row y of four planes by slot (plane & 3)
    float ang[4][kW3];                 // the same as loaded (live from the request to the arrival only)
    uint32_t gap[4];                   // gap bits of row y of the slot's plane
    uint32_t ngap;                     // gap bits of the plane last requested
    float ah[kH3];                     // the halo row of the plane last requested, at the halo columns
    float cu[kH3], su[kH3], cd[kH3], sd[kH3];   // rows y - 1 and y + 1 of the current plane at its updated columns
    long long e_acc;

    __device__ __forceinline__ float ld(int64_t off, int j) const
    {
        return *reinterpret_cast<const float*>(S + off + j * 256 + lane4);
    }
    __device__ __forceinline__ void st(int64_t off, int j, float v) const
    {
        *reinterpret_cast<float*>(S + off + j * 256 + lane4) = v;
    }
    __device__ __forceinline__ int64_t plane_off(int z) const { return orow + (int64_t)z * wplane; }
    __device__ __forceinline__ float2& xe(int buf, int slot, int k) const
    {
        return xch[((buf * (kNW3 + 2) + slot) * kH3 + k) * 64 + lane];
    }

    // row y of plane z (inside the grid or not) into slot SL; its gap bits
    template <int SL>
    __device__ __forceinline__ void request(int z)
    {
        if (z < 0 || z >= a.D) {
            ngap = 0u;
#pragma unroll
            for (int j = 0; j < kW3; ++j) ang[SL][j] = __builtin_nondeterministic_value(0.0f);
            return;
        }
        using CU = const __attribute__((address_space(4))) uint32_t;
        const uint64_t ad_ = (uint64_t)(cells + ((int64_t)z * a.H + y) * a.nbands + band);
        const CU* pc = (const CU*)((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)ad_) |
                                   ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(ad_ >> 32)) << 32));
        ngap = *pc;
        const int64_t off = plane_off(z);
        if (colmask == (1u << kW3) - 1u) {
#pragma unroll
            for (int j = 0; j < kW3; ++j) ang[SL][j] = ld(off, j);
        } else {
#pragma unroll
            for (int j = 0; j < kW3; ++j)
                ang[SL][j] = ((colmask >> j) & 1u) ? ld(off, j) : __builtin_nondeterministic_value(0.0f);
        }
    }

    // the requested row enters slot SL: (cos, sin) of the window, (0, 0) outside the grid (or for a plane outside)
    // (the (cos, sin) of every column are computed from whatever the slot holds and then cleared where needed,
    // behind scalar branches, so that the common case writes the slot once)
    template <int SL>
    __device__ __forceinline__ void arrive(int z)
    {
        gap[SL] = ngap;
#pragma unroll
        for (int j = 0; j < kW3; ++j) {
            const float t = a.q * ang[SL][j];
            c[SL][j] = cos_rev(t);
            s[SL][j] = sin_rev(t);
        }
        if (z < 0 || z >= a.D) {
#pragma unroll
            for (int j = 0; j < kW3; ++j) c[SL][j] = s[SL][j] = 0.0f;
        } else if (colmask != (1u << kW3) - 1u) {
#pragma unroll
            for (int j = 0; j < kW3; ++j)
                if (!((colmask >> j) & 1u)) c[SL][j] = s[SL][j] = 0.0f;
        }
    }

    // publishes the (cos, sin) of row y of the plane in slot SL at the columns its neighbour rows update there (the
    // columns of parity 1 - PX, PX this row's parity on that plane)
    template <int SL, int PX>
    __device__ __forceinline__ void publish(int buf) const
    {
#pragma unroll
        for (int k = 0; k < kH3; ++k) xe(buf, wslot, k) = make_float2(c[SL][2 * k + 2 - PX], s[SL][2 * k + 2 - PX]);
    }

    // the halo row of plane z at this wave's updated columns there (parity PX)
    template <int PX>
    __device__ __forceinline__ void request_halo(int z)
    {
        if (z < 0 || z >= a.D) return;
        const int64_t off = plane_off(z) + hoff;
        if (colmask == (1u << kW3) - 1u) {
#pragma unroll
            for (int k = 0; k < kH3; ++k) ah[k] = ld(off, 2 * k + PX + 1);
        } else {
#pragma unroll
            for (int k = 0; k < kH3; ++k)
                ah[k] = ((colmask >> (2 * k + PX + 1)) & 1u) ? ld(off, 2 * k + PX + 1)
                                                               : __builtin_nondeterministic_value(0.0f);
        }
    }
    template <int PX>
    __device__ __forceinline__ void arrive_halo(int z, int buf)
    {
        const bool inz = z >= 0 && z < a.D;
#pragma unroll
        for (int k = 0; k < kH3; ++k) {
            const float t = a.q * ah[k];
            float cv = cos_rev(t), sv = sin_rev(t);
            if (!inz || !((colmask >> (2 * k + PX + 1)) & 1u)) cv = sv = 0.0f;
            xe(buf, hslot, k) = make_float2(cv, sv);
            ah[k] = __builtin_nondeterministic_value(0.0f);
        }
    }

    // rows y - 1 and y + 1 of the plane in buffer buf, from the exchange
    __device__ __forceinline__ void read_nb(int buf)
    {
#pragma unroll
        for (int k = 0; k < kH3; ++k) {
            const float2 u = xe(buf, wslot - 1, k), d = xe(buf, wslot + 1, k);
            cu[k] = u.x;
            su[k] = u.y;
            cd[k] = d.x;
            sd[k] = d.y;
        }
    }

    // temperature entry of window column j in the block row `brow` (scalar load through the constant space); xb is
    // the band origin passed through an opaque copy, so that the column's block is computed here and not kept for
    // every column across the plane loop
    __device__ __forceinline__ TBand tband(int64_t brow, int xb, int j) const
    {
        using CU = const __attribute__((address_space(4))) uint32_t;
        const int xr = xb - 1 + j;
        const int x = xr < a.W ? xr : a.W - 1;     // a pair's second column may lie past the grid (not updated)
        const int bx = a.lb_w == 1 ? x : (int)__umulhi((uint32_t)x, a.lbw_inv);
        const uint64_t ad_ = (uint64_t)(tb + brow + bx);
        const CU* p = (const CU*)((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)ad_) |
                                  ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(ad_ >> 32)) << 32));
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = p[i];
        TBand t;
        __builtin_memcpy(&t, w, sizeof(TBand));
        return t;
    }

    // one Metropolis update of window column j of plane z (slot S0; back SP, front SN; rows y -+ 1 at index k)
    template <int S0, int SP, int SN>
    __device__ __forceinline__ int update(const TBand& T, int z, int64_t off, int j, int k, uint32_t wp, uint32_t wa)
    {
        const float Cx = ((((c[SP][j] + cu[k]) + c[S0][j - 1]) + c[S0][j + 1]) + cd[k]) + c[SN][j];
        const float Sy = ((((s[SP][j] + su[k]) + s[S0][j - 1]) + s[S0][j + 1]) + sd[k]) + s[SN][j];
        const float tp = u24(wp);
        const float ui = (float)(wa >> 8);
        const float angp = a.q * tp;
        const float cp = cos_rev(angp), sp = sin_rev(angp);
        const float co = c[S0][j], so = s[S0][j];
        const float X = fmaf(cp - co, Cx, (sp - so) * Sy);
        const float w24 = exp2_fast(fminf(fmaf(X, T.kappa, 24.0f), 25.0f));
        const bool tpos = __float_as_int(T.T) > 0;
        float r = tpos ? ui - w24 : -a.J * X;
        const float tol = tpos ? fmaf(w24, fmaf(fabsf(X), T.kb, T.band), 0.015625f) : a.delta_e;
        const bool need = fabsf(r) <= tol;
        if (__builtin_amdgcn_ballot_w64(need) != 0) {
            int xb = x0;
            asm volatile("" : "+s"(xb));
            const bool ex = exact3_site(S, off + j * 256 + lane4, wrow, wplane, xb - 1 + j, y, z, a.D, a.H, a.W, tp,
                                        ui, 2.0 * kPi * (double)a.q, (double)a.J, T.T);
            r = need ? (ex ? -1.0f : 1.0f) : r;
        }
        const bool acc = r < 0.0f;
        const float cf = acc ? cp : co, sf = acc ? sp : so;
        c[S0][j] = cf;
        s[S0][j] = sf;
        if (acc) st(off, j, tp);          // in place: a rejected proposal leaves the cell as it is
        return ENERGY ? fix24(-fmaf(cf, Cx, sf * Sy)) : 0;
    }

    // the colour of the launch on plane z (slot S0): the pairs of the updated columns, then the energy of the
    // colour-1 sample sites
    template <int S0, int YC>
    __device__ __forceinline__ void plane(int z)
    {
        constexpr int SP = (S0 + 3) & 3, SN = (S0 + 1) & 3;
        constexpr int PX = (YC + S0) & 1;              // (x + y + z + colour) even <=> x - x0 = PX mod 2
        const int64_t off = plane_off(z);
        const int64_t brow = (int64_t)bzc * a.bz_stride + byx;
        const uint32_t w3k1 = a.w3k1;
        const uint32_t base = ((uint32_t)z * (uint32_t)a.H + (uint32_t)y) * (uint32_t)a.Mw + (uint32_t)(x0 / 4);
        int xb = x0;
        asm volatile("" : "+s"(xb));
        int e = 0;
#pragma unroll
        for (int m = 0; m < kB3 / 4; ++m) {
            const int j0 = 4 * m + PX + 1, j1 = j0 + 2;
            const bool g0 = (gap[S0] >> j0) & 1u, g1 = (gap[S0] >> j1) & 1u;
            if (!(g0 || g1)) continue;
            const TBand T0 = tband(brow, xb, j0), T1 = tband(brow, xb, j1);
            const U4 w = philox_site(base + (uint32_t)m, w3k1, pl, rk);
            if (g0) e += update<S0, SP, SN>(T0, z, off, j0, 2 * m, w.x, w.y);
            if (g1) e += update<S0, SP, SN>(T1, z, off, j1, 2 * m + 1, w.z, w.w);
        }
        if (ENERGY) {
            const uint32_t smp = colmask & ~gap[S0];
#pragma unroll
            for (int k = 0; k < kH3; ++k) {
                const int j = 2 * k + PX + 1;
                if (!((smp >> j) & 1u)) continue;
                const float Cx = ((((c[SP][j] + cu[k]) + c[S0][j - 1]) + c[S0][j + 1]) + cd[k]) + c[SN][j];
                const float Sy = ((((s[SP][j] + su[k]) + s[S0][j - 1]) + s[S0][j + 1]) + sd[k]) + s[SN][j];
                e += fix24(-fmaf(c[S0][j], Cx, s[S0][j] * Sy));
            }
            e_acc += e;
        }
    }

    // one step (S0 = z & 3): plane z + 1 arrives and is published with the halo row of plane z + 1, plane z + 2
    // and the halo row of plane z + 2 are requested, rows y +- 1 of plane z come from the exchange, then plane z
    // is updated.  The caller ends the step with a barrier.
    template <int S0, int YC>
    __device__ __forceinline__ void step(int z)
    {
        constexpr int SN = (S0 + 1) & 3, S2 = (S0 + 2) & 3;
        constexpr int PX = (YC + S0) & 1, PXN = (YC + S0 + 1) & 1;
        arrive<SN>(z + 1);
        publish<SN, PXN>((z + 1) & 1);
        if (hoff != 0) {
            if (z + 1 < ze) arrive_halo<PXN>(z + 1, (z + 1) & 1);
            if (z + 2 < ze) request_halo<PX>(z + 2);
        }
        if (z + 2 <= ze) request<S2>(z + 2);
        read_nb(z & 1);
        plane<S0, YC>(z);
        if (++bzr == a.lb_d) {
            bzr = 0;
            ++bzc;
        }
    }

    // planes zs - 1 (slot 3) and zs (slot 0) in the window and published with the halo row of plane zs, plane zs + 1
    // and the halo row of plane zs + 1 requested; the caller then waits at the barrier
    template <int YC>
    __device__ __forceinline__ void start()
    {
        constexpr int PX0 = YC & 1, PX1 = (YC + 1) & 1;      // zs is a multiple of 4
        request<3>(zs - 1);
        arrive<3>(zs - 1);
        request<0>(zs);
        arrive<0>(zs);
        publish<0, PX0>(zs & 1);
        if (hoff != 0) {
            request_halo<PX0>(zs);
            arrive_halo<PX0>(zs, zs & 1);
            if (zs + 1 < ze) request_halo<PX1>(zs + 1);
        }
        request<1>(zs + 1);
    }

    // the wave's whole segment: the start, then one step per plane, each followed by the workgroup's barrier (the
    // exchange of plane z + 1 is complete at the barrier after step z)
    template <int YC>
    __device__ __forceinline__ void run()
    {
        start<YC>();
        __syncthreads();
        for (int zb = zs; zb < ze; zb += 4) {
            step<0, YC>(zb);
            __syncthreads();
            if (zb + 1 >= ze) break;
            step<1, YC>(zb + 1);
            __syncthreads();
            if (zb + 2 >= ze) break;
            step<2, YC>(zb + 2);
            __syncthreads();
            if (zb + 3 >= ze) break;
            step<3, YC>(zb + 3);
            __syncthreads();
        }
    }
};

// One launch is one colour of a sweep over all rows: workgroups of kNW3 waves (consecutive rows), work items
// (row tile, band, plane segment, group of realizations).
template <bool ENERGY>
__global__ __launch_bounds__(64 * kNW3) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep3(
    Lat3Args a, const uint32_t* __restrict__ cells, const TBand* __restrict__ tb, float* state,
    long long* __restrict__ epart)
{
    __shared__ float2 xch[2 * (kNW3 + 2) * kH3 * 64];
    // XCD-aware order: workgroup g runs on XCD g % 8; consecutive items (adjacent bands) go to the same XCD.
    const uint32_t N = (uint32_t)a.nrows * (uint32_t)a.nbands * (uint32_t)a.nzseg * (uint32_t)(a.Rp / 64);
    const uint32_t g = blockIdx.x, xcd = g & 7u, k = g >> 3;
    const uint32_t per = N >> 3, rem = N & 7u;
    const uint32_t item = xcd < rem ? xcd * (per + 1u) + k : rem * (per + 1u) + (xcd - rem) * per + k;
    if (item >= N) return;                           // the whole workgroup (item is the same for its waves)
    const uint32_t band = item % (uint32_t)a.nbands;
    uint32_t rest = item / (uint32_t)a.nbands;
    const uint32_t zseg = rest % (uint32_t)a.nzseg;
    rest /= (uint32_t)a.nzseg;
    const uint32_t tile = rest % (uint32_t)a.nrows;
    const uint32_t rg = rest / (uint32_t)a.nrows;
    const int64_t n_all = (int64_t)a.D * a.H * a.W;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    Lat3Loop la;
    la.D = a.D;
    la.H = a.H;
    la.W = a.W;
    la.nbands = a.nbands;
    la.Mw = a.Mw;
    la.lb_w = a.lb_w;
    la.lb_d = a.lb_d;
    la.lbw_inv = a.lbw_inv;
    la.w3k1 = ctr_word3(a.scene, TAG_SWEEP, (uint32_t)a.colour) ^ a.key1;
    la.q = a.q;
    la.J = a.J;
    la.delta_e = kDeltaE3 * a.J;
    la.bz_stride = (int64_t)a.nby * a.nbx;
    Wave3<ENERGY> w{la, cells, tb, reinterpret_cast<char*>(state) + (int64_t)rg * n_all * 256, xch};
    const int y0 = (int)tile * kNW3;
    w.y = y0 + wv;
    w.band = (int)band;
    w.x0 = (int)band * kB3;
    w.zs = (int)zseg * a.zseg;
    w.ze = w.zs + a.zseg < a.D ? w.zs + a.zseg : a.D;
    w.wslot = wv + 1;
    w.lane = threadIdx.x & 63u;
    w.lane4 = w.lane * 4u;
    const int lane = (int)(rg * 64 + w.lane);
    w.real = a.real_offset + (uint32_t)lane;
    const bool active = w.y < a.H;
    const int yc = (w.y + a.colour) & 1;
    // this wave's exchange slots start at zero in both buffers (rows outside the grid stay zero)
    const float2 zero2 = make_float2(0.0f, 0.0f);
    w.hoff = 0;
    w.hslot = 0;
#pragma unroll
    for (int kk = 0; kk < kH3; ++kk) w.xe(0, w.wslot, kk) = w.xe(1, w.wslot, kk) = zero2;
    if (wv == 0) {
#pragma unroll
        for (int kk = 0; kk < kH3; ++kk) w.xe(0, 0, kk) = w.xe(1, 0, kk) = zero2;
    }
    if (wv == kNW3 - 1) {
#pragma unroll
        for (int kk = 0; kk < kH3; ++kk) w.xe(0, kNW3 + 1, kk) = w.xe(1, kNW3 + 1, kk) = zero2;
    }
    w.e_acc = 0;
    __syncthreads();                                 // the zeroed slots before any publication
    if (active) {
        w.pl = philox_lane(w.real, a.sweep, a.key0, a.key1);
        w.rk = round_keys(a.key0, a.key1);
        w.wrow = (int64_t)a.W * 256;
        w.wplane = (int64_t)a.H * w.wrow;
        w.orow = ((int64_t)w.y * a.W + (w.x0 - 1)) * 256;
        w.colmask = 0u;
        for (int j = 0; j < kW3; ++j) {
            const int x = w.x0 - 1 + j;
            if (x >= 0 && x < a.W) w.colmask |= 1u << j;
        }
        w.colmask = __builtin_amdgcn_readfirstlane(w.colmask);
        w.bzc = w.zs / a.lb_d;
        w.bzr = w.zs % a.lb_d;
        w.byx = (int64_t)(w.y / a.lb_h) * a.nbx;
        if (wv == 0 && y0 > 0) {
            w.hoff = -w.wrow;
            w.hslot = 0;
        }
        if (wv == kNW3 - 1 && y0 + kNW3 < a.H) {
            w.hoff = w.wrow;
            w.hslot = kNW3 + 1;
        }
        // every wave of the workgroup passes the same number of barriers: one after the start and one per plane
        if (yc) w.template run<1>();
        else w.template run<0>();
    } else {
        for (int z = w.zs - 1; z < w.ze; ++z) __syncthreads();
    }
    if (ENERGY && active && lane < a.R)
        epart[(int64_t)lane * ((int64_t)a.H * a.nbands * a.nzseg) + ((int64_t)w.y * a.nbands + band) * a.nzseg +
              zseg] = w.e_acc;
}

// gap bits of each row's window columns (x0 - 1 .. x0 + kB3)
__global__ __launch_bounds__(256) void k_cells3(const uint8_t* __restrict__ mask, int64_t rows, int W, int nbands,
                                                 uint32_t* __restrict__ cells)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * nbands) return;
    const int64_t r = i / nbands;
    const int band = (int)(i % nbands);
    uint32_t g = 0u;
    for (int j = 0; j < kW3; ++j) {
        const int x = band * kB3 - 1 + j;
        if (x >= 0 && x < W && !mask[r * W + x]) g |= 1u << j;
    }
    cells[i] = g;
}

// Eq. (2) per 3D block: one workgroup per block, its sites in a fixed order per thread, a fixed-order reduction
constexpr int ST3_NT = 256;

__global__ __launch_bounds__(ST3_NT) void k_block_stats3(const float* __restrict__ t, const uint8_t* __restrict__ mask,
                                                          int64_t D, int64_t H, int64_t W, int lb_d, int lb_h,
                                                          int lb_w, int nbx, int nby, double two_pi_q, double J,
                                                          double* S, int* N, double* Ts, int* No)
{
    __shared__ double lds_d[ST3_NT / 64];
    __shared__ int lds_i[ST3_NT / 64];
    const int64_t b = blockIdx.x;
    const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby), bz = (int)(b / ((int64_t)nbx * nby));
    const int64_t z0 = (int64_t)bz * lb_d, y0 = (int64_t)by * lb_h, x0 = (int64_t)bx * lb_w;
    const int64_t nz = (z0 + lb_d < D ? lb_d : D - z0), ny = (y0 + lb_h < H ? lb_h : H - y0),
                  nx = (x0 + lb_w < W ? lb_w : W - x0);
    const int64_t HW = H * W;
    double s = 0.0, ts = 0.0;
    int n = 0, no = 0;
    for (int64_t i = threadIdx.x; i < nz * ny * nx; i += ST3_NT) {
        const int64_t z = z0 + i / (ny * nx), y = y0 + (i / nx) % ny, x = x0 + i % nx;
        const int64_t p = z * HW + y * W + x;
        if (!mask[p]) continue;
        const double tp = (double)t[p];
        ts += tp;
        ++no;
        if (x + 1 < W && mask[p + 1]) {
            s += -J * cos(two_pi_q * (tp - (double)t[p + 1]));
            ++n;
        }
        if (y + 1 < H && mask[p + W]) {
            s += -J * cos(two_pi_q * (tp - (double)t[p + W]));
            ++n;
        }
        if (z + 1 < D && mask[p + HW]) {
            s += -J * cos(two_pi_q * (tp - (double)t[p + HW]));
            ++n;
        }
    }
    s = block_sum<ST3_NT>(s, lds_d);
    ts = block_sum<ST3_NT>(ts, lds_d);
    n = block_sum<ST3_NT>(n, lds_i);
    no = block_sum<ST3_NT>(no, lds_i);
    if (threadIdx.x == 0) {
        S[b] = s;
        N[b] = n;
        Ts[b] = ts;
        No[b] = no;
    }
}

// start of the chains of a 3D scene (samples: t; gaps: the block mean of the samples, else the global mean, or a
// uniform from the start stream)
__global__ __launch_bounds__(256) void k_init3(Init3Args a)
{
    const int64_t HW = a.H * a.W, n_all = a.D * HW;
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (n >= n_all) return;
    const int64_t z = n / HW, y = (n / a.W) % a.H, x = n % a.W;
    float v;
    if (a.mask[n]) {
        v = a.t[n];
    } else if (a.mode == 1) {
        const int64_t b = ((z / a.lb_d) * a.nby + y / a.lb_h) * a.nbx + x / a.lb_w;
        v = a.No[b] > 0 ? (float)(a.Ts[b] / (double)a.No[b]) : *a.gmean;
    } else {
        const uint32_t Mw = (uint32_t)((a.W + 3) / 4);
        const uint32_t pair = (uint32_t)(z * a.H + y) * Mw + (uint32_t)(x >> 2);
        const uint32_t colour = (uint32_t)((x + y + z) & 1);
        const U4 w = philox4x32_10(pair, 0u, a.real_offset + (uint32_t)r, ctr_word3(a.scene, TAG_INIT, colour),
                                   a.key0, a.key1);
        v = u24(((x >> 1) & 1) ? w.z : w.x);
    }
    a.state[(int64_t)r * n_all + n] = v;
}

// fixed-point energy / J of the +x, +y, +z bonds of every site, per (part, realization)
constexpr int EN3_NT = 256;

__global__ __launch_bounds__(EN3_NT) void k_energy3_full(const float* __restrict__ state, int64_t D, int64_t H,
                                                          int64_t W, float q, long long* partial)
{
    __shared__ long long s_red[EN3_NT / 64];
    const int r = blockIdx.y;
    const int64_t HW = H * W, n_all = D * HW;
    const float* st = state + (int64_t)r * n_all;
    long long acc = 0;
    for (int64_t n = (int64_t)blockIdx.x * EN3_NT + threadIdx.x; n < n_all; n += (int64_t)gridDim.x * EN3_NT) {
        const int64_t z = n / HW, y = (n / W) % H, x = n % W;
        const float tn = st[n];
        float e = 0.0f;
        if (x + 1 < W) e -= cos_rev(q * (tn - st[n + 1]));
        if (y + 1 < H) e -= cos_rev(q * (tn - st[n + W]));
        if (z + 1 < D) e -= cos_rev(q * (tn - st[n + HW]));
        acc += fix24(e);
    }
    const long long tot = block_sum<EN3_NT>(acc, s_red);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = tot;
}

// one half-sweep of the periodic reference lattice (every site free, J = 1), one chain per temperature: a thread
// per same-colour pair of a row, the neighbours read from memory
__global__ __launch_bounds__(256) void k_ref3_half(float* state, const float* Tgrid, int L, uint32_t sweep, int colour,
                                                    float q, float delta_e, uint32_t key0, uint32_t key1,
                                                    double two_pi_q)
{
    const int chain = blockIdx.y;
    const int Mw = (L + 3) / 4;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t rows = (int64_t)L * L;
    if (p >= rows * Mw) return;
    const int64_t row = p / Mw;
    const int m = (int)(p - row * Mw);
    const int z = (int)(row / L), y = (int)(row % L);
    const int xa = 4 * m + ((y + z + colour) & 1);
    if (xa >= L) return;
    const int64_t L2 = (int64_t)L * L;
    float* st = state + (int64_t)chain * L2 * L;
    const float T = Tgrid[chain];
    const TBand tbd = make_tband(T, 1.0f, delta_e);
    const U4 w = philox4x32_10((uint32_t)p, sweep, (uint32_t)chain, ctr_word3(0u, TAG_REFLAT, (uint32_t)colour), key0,
                               key1);
    const int zb = (z + L - 1) % L, zf = (z + 1) % L, yu = (y + L - 1) % L, yd = (y + 1) % L;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int x = xa + 2 * h;
        if (x >= L) break;
        const int xl = (x + L - 1) % L, xr = (x + 1) % L;
        float nb[6];
        nb[0] = st[zb * L2 + (int64_t)y * L + x];
        nb[1] = st[z * L2 + (int64_t)yu * L + x];
        nb[2] = st[z * L2 + (int64_t)y * L + xl];
        nb[3] = st[z * L2 + (int64_t)y * L + xr];
        nb[4] = st[z * L2 + (int64_t)yd * L + x];
        nb[5] = st[zf * L2 + (int64_t)y * L + x];
        float Cx = 0.0f, Sy = 0.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const float an = q * nb[j];
            Cx += cos_rev(an);
            Sy += sin_rev(an);
        }
        const int64_t o = z * L2 + (int64_t)y * L + x;
        const float to = st[o];
        const float co = cos_rev(q * to), so = sin_rev(q * to);
        const float tpv = u24(h ? w.z : w.x);
        const uint32_t wa = h ? w.w : w.y;
        const float cp = cos_rev(q * tpv), sp = sin_rev(q * tpv);
        const float X = fmaf(cp - co, Cx, (sp - so) * Sy);
        int dec = filter32(X, (float)(wa >> 8), tbd, 1.0f, delta_e);
        if (dec < 0)
            dec = exact64_6(tpv, to, nb[0], nb[1], nb[2], nb[3], nb[4], nb[5], 63u, two_pi_q, 1.0, T, u24(wa)) ? 1 : 0;
        if (dec) st[o] = tpv;
    }
}

// per (part, chain): the sum over the part's sites of the energies of their +x, +y, +z bonds (periodic), FP64
__global__ __launch_bounds__(256) void k_ref3_energy(const float* __restrict__ state, int L, float q, double* partial)
{
    __shared__ double s_red[4];
    const int chain = blockIdx.y;
    const int64_t L2 = (int64_t)L * L, L3 = L2 * L;
    const float* st = state + (int64_t)chain * L3;
    double acc = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < L3; n += (int64_t)gridDim.x * 256) {
        const int64_t z = n / L2, y = (n / L) % L, x = n % L;
        const float tn = st[n];
        acc -= (double)cos_rev(q * (tn - st[z * L2 + y * L + (x + 1) % L]));
        acc -= (double)cos_rev(q * (tn - st[z * L2 + ((y + 1) % L) * L + x]));
        acc -= (double)cos_rev(q * (tn - st[((z + 1) % L) * L2 + y * L + x]));
    }
    const double tot = block_sum<256>(acc, s_red);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * gridDim.y + chain] = tot;   // layout [part][chain]
}

}  // namespace

int64_t lat3_blocks(int64_t D, int64_t H, int64_t W, int lb_d, int lb_h, int lb_w)
{
    return ((D + lb_d - 1) / lb_d) * ((H + lb_h - 1) / lb_h) * ((W + lb_w - 1) / lb_w);
}

hipError_t launch_block_stats3(const float* t, const uint8_t* mask, int64_t D, int64_t H, int64_t W, int lb_d,
                               int lb_h, int lb_w, double two_pi_q, double J, double* S, int* N, double* Ts, int* No,
                               hipStream_t s)
{
    const int nbx = (int)((W + lb_w - 1) / lb_w), nby = (int)((H + lb_h - 1) / lb_h);
    const int64_t B = lat3_blocks(D, H, W, lb_d, lb_h, lb_w);
    hipLaunchKernelGGL(k_block_stats3, dim3((unsigned)B), dim3(ST3_NT), 0, s, t, mask, D, H, W, lb_d, lb_h, lb_w, nbx,
                       nby, two_pi_q, J, S, N, Ts, No);
    return hipGetLastError();
}

hipError_t launch_init3(const Init3Args& a, hipStream_t s)
{
    const int64_t n_all = a.D * a.H * a.W;
    hipLaunchKernelGGL(k_init3, dim3((unsigned)((n_all + 255) / 256), (unsigned)a.R), dim3(256), 0, s, a);
    return hipGetLastError();
}

int energy3_parts(int64_t D, int64_t H, int64_t W)
{
    const int64_t n = D * H * W;
    const int64_t p = (n + EN3_NT * 16 - 1) / (EN3_NT * 16);
    return (int)(p < 1 ? 1 : (p > 256 ? 256 : p));
}

hipError_t launch_energy3_full(const float* state, int64_t D, int64_t H, int64_t W, int R, float q, long long* partial,
                               int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy3_full, dim3((unsigned)nparts, (unsigned)R), dim3(EN3_NT), 0, s, state, D, H, W, q,
                       partial);
    return hipGetLastError();
}

hipError_t launch_cells3(const uint8_t* mask, int64_t D, int64_t H, int64_t W, int nbands, uint32_t* cells,
                         hipStream_t s)
{
    const int64_t rows = D * H;
    hipLaunchKernelGGL(k_cells3, dim3((unsigned)((rows * nbands + 255) / 256)), dim3(256), 0, s, mask, rows, (int)W,
                       nbands, cells);
    return hipGetLastError();
}

hipError_t launch_sweep3(const Lat3Args& a, const uint32_t* cells, const TBand* tb, float* state, long long* epart,
                         hipStream_t s)
{
    const int64_t N = (int64_t)a.nrows * a.nbands * a.nzseg * (a.Rp / 64);
    if (N <= 0) return hipSuccess;
    const dim3 grid((unsigned)N);
    if (epart) hipLaunchKernelGGL((k_sweep3<true>), grid, dim3(64 * kNW3), 0, s, a, cells, tb, state, epart);
    else hipLaunchKernelGGL((k_sweep3<false>), grid, dim3(64 * kNW3), 0, s, a, cells, tb, state, epart);
    return hipGetLastError();
}

hipError_t launch_ref3_half(float* state, const float* Tgrid, int nT, int L, uint32_t sweep, int colour, float q,
                            float delta_e, uint32_t key0, uint32_t key1, double two_pi_q, hipStream_t s)
{
    const int64_t np = (int64_t)L * L * ((L + 3) / 4);
    hipLaunchKernelGGL(k_ref3_half, dim3((unsigned)((np + 255) / 256), (unsigned)nT), dim3(256), 0, s, state, Tgrid, L,
                       sweep, colour, q, delta_e, key0, key1, two_pi_q);
    return hipGetLastError();
}

int ref3_energy_parts(int L)
{
    const int64_t n = (int64_t)L * L * L;
    const int64_t p = (n + 4095) / 4096;
    return (int)(p < 1 ? 1 : (p > 128 ? 128 : p));
}

hipError_t launch_ref3_energy(const float* state, int L, int nT, float q, double* partial, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_ref3_energy, dim3((unsigned)nparts, (unsigned)nT), dim3(256), 0, s, state, L, q, partial);
    return hipGetLastError();
}

}  // namespace mpr
