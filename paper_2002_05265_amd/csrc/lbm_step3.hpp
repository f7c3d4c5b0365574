// Three time steps per pass over one strip of a grid (temporal blocking with two LDS rings), shared
// by the plain three-step kernel and the batched one.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_cell.hpp"
#include "lbm_internal.hpp"
#include "lbm_step2.hpp"

namespace lbm {

// Steps `step`, `step` + 1 and `step` + 2 of the strip of columns x0 .. x0 + W - 1 and rows
// ys .. ye - 1 of grid g: pulls from src, writes to dst, collides with coll(h, m).  The first step
// covers the strip plus two halo rows and columns on each side and keeps its post-collision values
// in ring1 (RING + 2 rows of W + 4 columns), the second covers one halo row and column on each side
// and pulls from ring1 into ring2 (RING + 2 rows of W + 2 columns), the third pulls from ring2 and
// writes to memory.  Per three steps each population is read from and written to memory once.  In a
// pass the three steps work on rows two, one and zero rows ahead of the pass base yb (each needs
// the rows above and below from the step before), so a pass has two block barriers, as the
// two-step pass.  Every node is computed by the same arithmetic as in k_step and the rings hold the
// values in the storage type, so the result is bit-identical to three launches of k_step.  VIA_L2
// selects L1-bypassing loads, NT streaming stores (as in strip_two_steps).  Requires nx, ny >= 2
// (one conditional wrap of rows and columns) and strip rows >= 1.  Called by all 64 NW threads of a
// workgroup (NW waves: 4, or 8 with one row per wave and pass for a ring of 8 rows); the last wave
// also collides the first step's halo columns, the one before it the second step's.
template <int RING, int W, bool VIA_L2 = false, bool NT = true, int NW = 4, typename S, typename R, typename Coll>
__device__ __forceinline__ void strip_three_steps(S (&ring1)[9][RING + 2][W + 4], S (&ring2)[9][RING + 2][W + 2],
                                                  const S* __restrict__ src, S* __restrict__ dst, const Geom& g,
                                                  const Ref<R>& ref, int x0, int ys, int ye, int step,
                                                  int* __restrict__ blowup, Coll&& coll) {
    constexpr int NR = RING + 2;
    constexpr int WPR = W / 64;     // waves per row of the strip
    constexpr int RPW = NW / WPR;   // rows the block covers at once
    constexpr int KR = RING / RPW;  // rows per wave and pass
    constexpr int H1 = NW - 1, H2 = NW - 2;  // the waves that take the first / second step's halo
    static_assert(RING % RPW == 0 && 4 * RING <= 64, "ring rows: a multiple of the block's rows, at most 16");
    const int lane = (int)(threadIdx.x & 63u);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int cg = wave % WPR, rl = wave / WPR;
    const int w = min(W, g.nx - x0);  // output columns of this strip
    const int col = cg * 64 + lane;   // this lane's column in the strip
    const bool in1 = col < w;
    const int lc1 = col + 2, lc2 = col + 1;  // and in ring1 / ring2
    constexpr unsigned E = sizeof(S);
    unsigned xo0, xom, xop;
    {
        int x = x0 + col;
        x = x >= g.nx ? x - g.nx : x;
        xo0 = (unsigned)x * E;
        xom = (unsigned)(x == 0 ? g.nx - 1 : x - 1) * E;
        xop = (unsigned)(x == g.nx - 1 ? 0 : x + 1) * E;
    }
    auto wrap_row = [&](int a) { return a < 0 ? a + g.ny : (a >= g.ny ? a - g.ny : a); };
    // first-step pull loads of row a (wave-uniform) at the lane's own column: scalar row
    // pointers plus the lane's fixed column offsets (taken afresh so that their widening to 64
    // bits stays next to the loads)
    auto load_own = [&](int a, R (&h)[9]) {
        const int yw = wrap_row(a);
        const long long r0 = (long long)yw * g.nx;
        const long long rm = yw == 0 ? (long long)(g.ny - 1) * g.nx : r0 - g.nx;
        const long long rp = yw == g.ny - 1 ? 0 : r0 + g.nx;
        unsigned o0 = xo0, om = xom, op = xop;
        asm("" : "+v"(o0), "+v"(om), "+v"(op));
        auto at = [&](int q, long long r, unsigned xo) { return byte_off(wave_uniform(src + q * g.plane + r), xo); };
        auto get = [&](const S* p) {
            if constexpr (VIA_L2) return ld_l2(p); else return ld(p);
        };
        h[0] = R(get(at(0, r0, o0)));
        h[1] = R(get(at(1, r0, om)));
        h[2] = R(get(at(2, rm, o0)));
        h[3] = R(get(at(3, r0, op)));
        h[4] = R(get(at(4, rp, o0)));
        h[5] = R(get(at(5, rm, om)));
        h[6] = R(get(at(6, rm, op)));
        h[7] = R(get(at(7, rp, op)));
        h[8] = R(get(at(8, rp, om)));
    };
    // first-step pull loads of row a (per lane) at ring1 column c1 (grid column x0 - 2 + c1)
    auto load_any = [&](int a, int c1, R (&h)[9]) {
        const int x = x0 - 2 + c1;
        const int xw = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
        if constexpr (VIA_L2)
            pull_load_l2(src, g.plane, neighbours(xw, wrap_row(a), g.nx, g.ny), h);
        else
            pull_load(src, g.plane, neighbours(xw, wrap_row(a), g.nx, g.ny), h);
    };
    // ring1 column of halo lane code k (0..3): grid columns x0 - 2, x0 - 1, x0 + w, x0 + w + 1
    auto halo1_col = [&](int k) { return k < 2 ? k : w + k; };
    auto wrap = [](int t) { return t < 0 ? t + NR : (t >= NR ? t - NR : t); };
    // ring slots: row a is in ring1 slot (a - ys + 2) mod NR and in ring2 slot (a - ys + 1) mod NR
    auto finish1 = [&](int slot, int c1, R (&h)[9]) {
        double rho_d;
        const Macro<R> m = macro_of<S>(h, ref, rho_d);
        flag_bad(!(rho_d > 0.0), blowup, step);
        coll(h, m);
#pragma unroll
        for (int i = 0; i < 9; ++i) ring1[i][slot][c1] = to_store<S>(h[i]);
    };
    // second step of the node at ring2 column c2 whose row's ring1 slot is s1 (unwrapped), into
    // ring2 slot s2
    auto second = [&](int s1, int c2, int s2) {
        R h[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = R(ring1[i][wrap(s1 - cy(i))][c2 + 1 - cx(i)]);
        double rho_d;
        const Macro<R> m = macro_of<S>(h, ref, rho_d);
        flag_bad(!(rho_d > 0.0), blowup, step + 1);
        coll(h, m);
#pragma unroll
        for (int i = 0; i < 9; ++i) ring2[i][s2][c2] = to_store<S>(h[i]);
    };

    R hn[KR][9];
    R hh[9];
    // loads of the first step of a pass with base yb: rows yb + 2 .. min(yb + RING + 1, ye + 1);
    // wave 3 also takes the four halo columns of those rows (four lanes per row)
    auto prefetch = [&](int yb) {
        const int top = min(yb + RING + 1, ye + 1);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 2 + rl + RPW * k;
            if (a <= top && in1) load_own(a, hn[k]);
        }
        if (wave == H1) {
            const int a = yb + 2 + (lane >> 2);
            if (a <= top && lane < 4 * RING) load_any(a, halo1_col(lane & 3), hh);
        }
    };

    // prologue, first step: rows ys - 2 .. ys + 1 (ring1 slots 0..3) with their halo columns
    {
        constexpr int KP = (4 + RPW - 1) / RPW;
        R hp[KP][9];
        R hq[9];
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (in1 && rl + RPW * k < 4) load_own(ys - 2 + rl + RPW * k, hp[k]);
        if (wave == H1 && lane < 16) load_any(ys - 2 + (lane >> 2), halo1_col(lane & 3), hq);
        prefetch(ys);
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (in1 && rl + RPW * k < 4) finish1(rl + RPW * k, lc1, hp[k]);
        if (wave == H1 && lane < 16) finish1(lane >> 2, halo1_col(lane & 3), hq);
    }
    __syncthreads();
    // prologue, second step: rows ys - 1 and ys (ring2 slots 0, 1; ring1 slots 1, 2) with their
    // halo columns (wave H2, lanes 0..3)
    {
        if (rl < 2 && in1) second(1 + rl, lc2, rl);
        if (wave == H2 && lane < 4) second(1 + (lane >> 1), (lane & 1) ? w + 1 : 0, lane >> 1);
    }
    __syncthreads();

    for (int yb = ys; yb < ye; yb += RING) {
        const int top1 = min(yb + RING + 1, ye + 1);  // first step: rows yb + 2 .. top1
        const int top2 = min(yb + RING, ye);          // second step: rows yb + 1 .. top2
        const int sb1 = (yb - ys + 2) % NR;           // ring1 slot of row yb
        const int sb2 = (yb - ys + 1) % NR;           // ring2 slot of row yb
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 2 + rl + RPW * k;
            if (a <= top1 && in1) finish1(wrap(sb1 + 2 + rl + RPW * k), lc1, hn[k]);
        }
        if (wave == H1) {
            const int a = yb + 2 + (lane >> 2);
            if (a <= top1 && lane < 4 * RING) finish1(wrap(sb1 + 2 + (lane >> 2)), halo1_col(lane & 3), hh);
        }
        __syncthreads();
        if (yb + RING < ye) prefetch(yb + RING);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int off = 1 + rl + RPW * k;  // row yb + off
            if (yb + off <= top2 && in1) second(sb1 + off, lc2, wrap(sb2 + off));
        }
        if (wave == H2) {
            const int off = 1 + (lane >> 1);
            if (yb + off <= top2 && lane < 2 * RING) second(sb1 + off, (lane & 1) ? w + 1 : 0, wrap(sb2 + off));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int y = yb + rl + RPW * k;
            if (y < ye && in1) {
                const int s0 = sb2 + rl + RPW * k;  // ring2 slot of row y, before wrapping
                R h[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) h[i] = R(ring2[i][wrap(s0 - cy(i))][lc2 - cx(i)]);
                double rho_d;
                const Macro<R> m = macro_of<S>(h, ref, rho_d);
                flag_bad(!(rho_d > 0.0), blowup, step + 2);
                coll(h, m);
                const long long r = (long long)y * g.nx + x0;
                unsigned o = (unsigned)col * E;
                asm("" : "+v"(o));
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st<S, NT>(byte_off(wave_uniform(dst + i * g.plane + r), o), to_store<S>(h[i]));
            }
        }
    }
}

}  // namespace lbm

namespace lbm {

// Three steps per pass over a strip of WP output columns whose halo columns fit the wave: lane l
// takes column x0 - 2 + l in all three steps, the first step on lanes 0 .. WP + 3 (the strip and two
// halo columns each side), the second on lanes 1 .. WP + 2, the third on lanes 2 .. WP + 1, which
// write; there are no halo passes.  With WP = 48 in FP64 an output row segment is three whole
// 128-byte lines and the rings take 44 KiB with a ring of 4 rows (three workgroups per CU against two
// for 64 columns), 74 KiB with a ring of 8 (two workgroups of 8 waves).
// Same rows, ring slots and barriers as strip_three_steps; one wave per row, NW waves (4, or 8 with
// a ring of 8 rows).  VIA_L2 selects L1-bypassing loads, NT streaming stores.
template <int RING, int WP, bool VIA_L2 = false, bool NT = true, int NW = 4, typename S, typename R, typename Coll>
__device__ __forceinline__ void strip_three_steps_narrow(S (&ring1)[9][RING + 2][WP + 4],
                                                         S (&ring2)[9][RING + 2][WP + 3],
                                                         const S* __restrict__ src, S* __restrict__ dst,
                                                         const Geom& g, const Ref<R>& ref, int x0, int ys, int ye,
                                                         int step, int* __restrict__ blowup, Coll&& coll) {
    constexpr int NR = RING + 2;
    constexpr int KR = RING / NW;  // rows per wave and pass
    static_assert(RING % NW == 0 && WP + 4 <= 64, "ring rows: a multiple of the waves; the strip and its halo fit a wave");
    const int lane = (int)(threadIdx.x & 63u);
    const int rl = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = min(WP, g.nx - x0);            // output columns of this strip
    const bool on1 = lane < w + 4;               // first step: columns x0 - 2 .. x0 + w + 1
    const bool on2 = lane >= 1 && lane <= w + 2;  // second step: x0 - 1 .. x0 + w
    const bool on3 = lane >= 2 && lane <= w + 1;  // third step: x0 .. x0 + w - 1
    constexpr unsigned E = sizeof(S);
    unsigned xo0, xom, xop;
    {
        int x = x0 - 2 + lane;
        x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
        xo0 = (unsigned)x * E;
        xom = (unsigned)(x == 0 ? g.nx - 1 : x - 1) * E;
        xop = (unsigned)(x == g.nx - 1 ? 0 : x + 1) * E;
    }
    auto wrap_row = [&](int a) { return a < 0 ? a + g.ny : (a >= g.ny ? a - g.ny : a); };
    auto load_own = [&](int a, R (&h)[9]) {
        const int yw = wrap_row(a);
        const long long r0 = (long long)yw * g.nx;
        const long long rm = yw == 0 ? (long long)(g.ny - 1) * g.nx : r0 - g.nx;
        const long long rp = yw == g.ny - 1 ? 0 : r0 + g.nx;
        unsigned o0 = xo0, om = xom, op = xop;
        asm("" : "+v"(o0), "+v"(om), "+v"(op));
        auto at = [&](int q, long long r, unsigned xo) { return byte_off(wave_uniform(src + q * g.plane + r), xo); };
        auto get = [&](const S* p) {
            if constexpr (VIA_L2) return ld_l2(p); else return ld(p);
        };
        h[0] = R(get(at(0, r0, o0)));
        h[1] = R(get(at(1, r0, om)));
        h[2] = R(get(at(2, rm, o0)));
        h[3] = R(get(at(3, r0, op)));
        h[4] = R(get(at(4, rp, o0)));
        h[5] = R(get(at(5, rm, om)));
        h[6] = R(get(at(6, rm, op)));
        h[7] = R(get(at(7, rp, op)));
        h[8] = R(get(at(8, rp, om)));
    };
    auto wrap = [](int t) { return t < 0 ? t + NR : (t >= NR ? t - NR : t); };
    auto finish1 = [&](int slot, R (&h)[9]) {
        double rho_d;
        const Macro<R> m = macro_of<S>(h, ref, rho_d);
        flag_bad(!(rho_d > 0.0), blowup, step);
        coll(h, m);
#pragma unroll
        for (int i = 0; i < 9; ++i) ring1[i][slot][lane] = to_store<S>(h[i]);
    };
    auto second = [&](int s1, int s2) {
        R h[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = R(ring1[i][wrap(s1 - cy(i))][lane - cx(i)]);
        double rho_d;
        const Macro<R> m = macro_of<S>(h, ref, rho_d);
        flag_bad(!(rho_d > 0.0), blowup, step + 1);
        coll(h, m);
#pragma unroll
        for (int i = 0; i < 9; ++i) ring2[i][s2][lane] = to_store<S>(h[i]);
    };
    R hn[KR][9];
    auto prefetch = [&](int yb) {
        const int top = min(yb + RING + 1, ye + 1);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 2 + rl + NW * k;
            if (a <= top && on1) load_own(a, hn[k]);
        }
    };
    // prologue: first step on rows ys - 2 .. ys + 1 (ring1 slots 0..3), second on ys - 1, ys
    {
        R hp[9];
        if (on1 && rl < 4) load_own(ys - 2 + rl, hp);
        prefetch(ys);
        if (on1 && rl < 4) finish1(rl, hp);
    }
    __syncthreads();
    if (rl < 2 && on2) second(1 + rl, rl);
    __syncthreads();
    for (int yb = ys; yb < ye; yb += RING) {
        const int top1 = min(yb + RING + 1, ye + 1);
        const int top2 = min(yb + RING, ye);
        const int sb1 = (yb - ys + 2) % NR;
        const int sb2 = (yb - ys + 1) % NR;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 2 + rl + NW * k;
            if (a <= top1 && on1) finish1(wrap(sb1 + 2 + rl + NW * k), hn[k]);
        }
        __syncthreads();
        if (yb + RING < ye) prefetch(yb + RING);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int off = 1 + rl + NW * k;
            if (yb + off <= top2 && on2) second(sb1 + off, wrap(sb2 + off));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int y = yb + rl + NW * k;
            if (y < ye && on3) {
                const int s0 = sb2 + rl + NW * k;
                R h[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) h[i] = R(ring2[i][wrap(s0 - cy(i))][lane - cx(i)]);
                double rho_d;
                const Macro<R> m = macro_of<S>(h, ref, rho_d);
                flag_bad(!(rho_d > 0.0), blowup, step + 2);
                coll(h, m);
                const long long r = (long long)y * g.nx;
                unsigned o = xo0;
                asm("" : "+v"(o));
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st<S, NT>(byte_off(wave_uniform(dst + i * g.plane + r), o), to_store<S>(h[i]));
            }
        }
    }
}

}  // namespace lbm
