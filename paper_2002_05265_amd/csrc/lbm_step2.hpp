// Two time steps per pass over one strip of a grid (temporal blocking), shared by the plain
// two-step kernel and the batched one.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_cell.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// Two steps per pass over memory (temporal blocking).  A block owns a strip of columns and `hs`
// rows and walks down it RING rows at a time: the first step's post-collision values of the
// strip plus one halo column on each side are kept in a ring of RING + 2 rows in LDS, and the
// second step pulls from that ring and writes to memory.  Per two steps each population is read
// from and written to memory once, against twice for two single steps; the halo columns and the
// two rows above and below the strip are collided twice (by both strips that need them).  Every
// node is computed by the same arithmetic as in k_step and the ring holds the values in the
// storage type, so the result is bit-identical to two launches of k_step.
//
// Strips are 64 columns wide (128 for some models, see strip_width in lbm_core.hip), so every
// output row segment is whole 256-byte lines; lane l of a wave takes column x0 + 64 c + l of its
// column group c, and one wave collides the two halo columns of the pass's rows in an extra pass.
// (A 62-column strip with the halo columns in lanes 0 and 63 saves that pass, but its stores
// start mid-line and two strips write parts of the same lines: measured 0.6x as fast.)
constexpr int kStripW = 64;

// Loads that bypass the CU's L1 (agent scope) and are served by the XCD's L2: what the batched
// kernel's workgroups read was written by other workgroups of the same XCD during the launch.
template <typename S>
__device__ __forceinline__ S ld_l2(const S* p) {
    if constexpr (sizeof(S) == 2) {
        const unsigned short v = __hip_atomic_load(reinterpret_cast<const unsigned short*>(p), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        return __builtin_bit_cast(S, v);
    } else {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// pull_load (f_i(x) = stored_i(x - xi_i)) through ld_l2.
template <typename S, typename R>
__device__ __forceinline__ void pull_load_l2(const S* __restrict__ src, long long plane, const Nbr& n, R (&h)[9]) {
    constexpr unsigned E = sizeof(S);
    const unsigned r0 = n.r0 * E, rm = n.rm * E, rp = n.rp * E;
    const unsigned x0 = n.x * E, xm = n.xm * E, xp = n.xp * E;
    h[0] = R(ld_l2(plane_at(src, plane, 0, r0 + x0)));
    h[1] = R(ld_l2(plane_at(src, plane, 1, r0 + xm)));
    h[2] = R(ld_l2(plane_at(src, plane, 2, rm + x0)));
    h[3] = R(ld_l2(plane_at(src, plane, 3, r0 + xp)));
    h[4] = R(ld_l2(plane_at(src, plane, 4, rp + x0)));
    h[5] = R(ld_l2(plane_at(src, plane, 5, rm + xm)));
    h[6] = R(ld_l2(plane_at(src, plane, 6, rm + xp)));
    h[7] = R(ld_l2(plane_at(src, plane, 7, rp + xp)));
    h[8] = R(ld_l2(plane_at(src, plane, 8, rp + xm)));
}

// A pointer that is the same on every lane of the wave, made explicit (scalar registers, global
// address space), and an access at a per-lane 32-bit byte offset from it: the global load /
// store then takes its scalar-base form and needs no per-lane 64-bit address arithmetic.
template <typename T> struct Global { typedef __attribute__((address_space(1))) T type; };

template <typename T>
__device__ __forceinline__ T* wave_uniform(T* p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T*)(typename Global<T>::type*)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* byte_off(T* p, unsigned off) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + off);
}

// Steps `step` and `step` + 1 of the strip of columns x0 .. x0 + W - 1 and rows ys .. ye - 1
// of grid g: pulls from src, writes to dst, collides with coll(h, m).  Called by all 256 threads
// of a workgroup (it contains block barriers); ring is the workgroup's LDS ring.  VIA_L2 selects
// L1-bypassing loads, NT streaming stores; with MID the strip's nodes after the first step are
// also written to mid (the state a single step would have written).  Blow-up records go to
// *blowup (steps step and step + 1).
template <int RING, int W, bool VIA_L2, bool NT, bool MID = false, typename S, typename R, typename Coll>
__device__ __forceinline__ void strip_two_steps(S (&ring)[9][RING + 2][W + 2], const S* __restrict__ src,
                                                S* __restrict__ dst, const Geom& g, const Ref<R>& ref, int x0,
                                                int ys, int ye, int step, int* __restrict__ blowup, Coll&& coll,
                                                S* __restrict__ mid = nullptr) {
    constexpr int NR = RING + 2;
    constexpr int WPR = W / 64;        // waves per row of the strip
    constexpr int RPW = 4 / WPR;       // rows the block covers at once
    constexpr int KR = RING / RPW;     // rows per wave and pass
    const int lane = (int)(threadIdx.x & 63u);
    // the wave index is the same on every lane: read it as such, so that rows, ring slots and
    // row offsets below are scalar arithmetic and not repeated per lane
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int cg = wave % WPR, rl = wave / WPR;
    const int w = min(W, g.nx - x0);           // output columns of this strip
    const int col = cg * 64 + lane;            // this lane's column in the strip
    const int lc = col + 1;                    // and in the ring
    const bool in1 = col < w;
    // byte offsets of the lane's column and its two neighbours (wrapped), fixed for the strip
    constexpr unsigned E = sizeof(S);
    unsigned xo0, xom, xop;
    {
        int x = x0 + col;
        x = x >= g.nx ? x - g.nx : x;
        xo0 = (unsigned)x * E;
        xom = (unsigned)(x == 0 ? g.nx - 1 : x - 1) * E;
        xop = (unsigned)(x == g.nx - 1 ? 0 : x + 1) * E;
    }

    // first step at row a (ys - 1 <= a <= ye, unwrapped) and ring column cc (column
    // x0 - 1 + cc, wrapped): the pull loads, then the collision into the ring
    auto load = [&](int a, int cc, R (&h)[9]) {
        const int x = x0 - 1 + cc;
        const int yw = a < 0 ? a + g.ny : (a >= g.ny ? a - g.ny : a);
        const int xw = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
        if constexpr (VIA_L2)
            pull_load_l2(src, g.plane, neighbours(xw, yw, g.nx, g.ny), h);
        else
            pull_load(src, g.plane, neighbours(xw, yw, g.nx, g.ny), h);
    };
    // first step at the lane's own column of row a (the same row on the whole wave): the row
    // part of each address is a scalar pointer, the column part the lane's fixed offset
    auto load_own = [&](int a, R (&h)[9]) {
        const int yw = a < 0 ? a + g.ny : (a >= g.ny ? a - g.ny : a);
        const long long r0 = (long long)yw * g.nx;
        const long long rm = yw == 0 ? (long long)(g.ny - 1) * g.nx : r0 - g.nx;
        const long long rp = yw == g.ny - 1 ? 0 : r0 + g.nx;
        // the lane offsets are taken afresh here (an empty asm) so that their widening to 64 bits
        // is not hoisted out of the loop, which would cost a 64-bit vector add per load
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
    // ring slot of row a is (a - ys + 1) mod NR; within a pass it is reached from the pass's slot
    // base sb = (yb - ys + 1) mod NR by an offset in [-1, NR), so one conditional wrap suffices
    auto wrap = [](int t) { return t < 0 ? t + NR : (t >= NR ? t - NR : t); };
    // a: the node's row (for the intermediate state, which takes the strip's own nodes only)
    auto finish = [&](int slot, int cc, int a, R (&h)[9]) {
        double rho_d;
        const Macro<R> m = macro_of<S>(h, ref, rho_d);
        flag_bad(!(rho_d > 0.0), blowup, step);
        coll(h, m);
#pragma unroll
        for (int i = 0; i < 9; ++i) ring[i][slot][cc] = to_store<S>(h[i]);
        if constexpr (MID) {
            if (cc >= 1 && cc <= w && a >= ys && a < ye)
                store_cell<S, R, NT>(mid, g.plane, (unsigned)a * (unsigned)g.nx + (unsigned)(x0 + cc - 1), h);
        }
    };
    // Rows of a pass starting at yb: wave v takes rows yb + 1 + rl + RPW k of its column group,
    // and wave 3 also the halo columns of rows yb + 1 .. (two lanes per row).  The loads of the
    // next pass are issued before the second step of the current one, so their latency overlaps
    // it.
    R hn[KR][9];
    R hh[9];
    auto prefetch = [&](int yb) {
        const int top = min(yb + RING, ye);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 1 + rl + RPW * k;
            if (a <= top && in1) load_own(a, hn[k]);
        }
        if (wave == 3) {
            const int a = yb + 1 + (lane >> 1);
            if (a <= top) load(a, (lane & 1) ? w + 1 : 0, hh);
        }
    };

    // rows ys - 1 and ys (row lanes 0 and 1) and their halo columns, their loads issued together
    // with those of the first pass.  With one wave per row, wave 2 takes the four halo nodes and
    // every wave makes one collision call (the kernel stays one collision shorter); with two,
    // every wave has a row and wave 3 takes the halo nodes as well.
    // (rows ys - 1 and ys sit in slots 0 and 1)
    if constexpr (WPR == 1) {
        R h[9];
        const int r = wave < 2 ? wave : lane >> 1;
        const int cc = wave < 2 ? lc : ((lane & 1) ? w + 1 : 0);
        const bool act = wave < 2 ? in1 : (wave == 2 && lane < 4);
        if (act) load(ys - 1 + r, cc, h);
        prefetch(ys);
        if (act) finish(r, cc, ys - 1 + r, h);
    } else {
        R h[9], hp[9];
        const bool act = rl < 2 && in1;
        const bool acth = wave == 3 && lane < 4;
        const int rh = lane >> 1, ch = (lane & 1) ? w + 1 : 0;
        if (act) load(ys - 1 + rl, lc, h);
        if (acth) load(ys - 1 + rh, ch, hp);
        prefetch(ys);
        if (act) finish(rl, lc, ys - 1 + rl, h);
        if (acth) finish(rh, ch, ys - 1 + rh, hp);
    }
    for (int yb = ys; yb < ye; yb += RING) {
        const int top = min(yb + RING, ye);   // first step of rows yb + 1 .. top
        const int sb = (yb - ys + 1) % NR;    // slot of row yb (wave-uniform)
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int a = yb + 1 + rl + RPW * k;
            if (a <= top && in1) finish(wrap(sb + 1 + rl + RPW * k), lc, a, hn[k]);
        }
        if (wave == 3) {
            const int a = yb + 1 + (lane >> 1);
            if (a <= top) finish(wrap(sb + 1 + (lane >> 1)), (lane & 1) ? w + 1 : 0, a, hh);
        }
        __syncthreads();
        if (yb + RING < ye) prefetch(yb + RING);
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int y = yb + rl + RPW * k;
            if (y < ye && in1) {
                const int s0 = sb + rl + RPW * k;  // slot of row y, before wrapping
                R h[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) h[i] = R(ring[i][wrap(s0 - cy(i))][lc - cx(i)]);
                double rho_d;
                const Macro<R> m = macro_of<S>(h, ref, rho_d);
                flag_bad(!(rho_d > 0.0), blowup, step + 1);
                coll(h, m);
                const long long r = (long long)y * g.nx + x0;
                unsigned o = (unsigned)col * E;
                asm("" : "+v"(o));  // as in load_own
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st<S, NT>(byte_off(wave_uniform(dst + i * g.plane + r), o), to_store<S>(h[i]));
            }
        }
        __syncthreads();
    }
}

}  // namespace lbm
