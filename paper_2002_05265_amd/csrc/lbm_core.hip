// liblbm: fused periodic D2Q9 stream-and-collide for gfx950, and the C ABI declared in lbm.h.
//
// Data layout in HBM: two copies of nine population planes, plane q of copy c at
//   base + (c * 9 + q) * plane elements, plane = nx * ny rounded up to 256 bytes,
// each plane [y][x] with x fastest.  A wavefront (64 lanes) handles 64 consecutive x of one
// row, so every population load and store of a wave is one contiguous 64-element segment.
//
// Time stepping (eq. StreamCollide) is a pull scheme: the buffer of copy `cur` holds the
// post-collision populations f*(., n-1); a step gathers f_i(x, n) = f*_i(x - xi_i, n-1) with
// periodic wrap, collides in registers and writes f*(x, n) to the other copy.  Streaming is a
// pure permutation of stored values, so it is exact.  The initial state is written
// pre-streamed backwards (stored_i(x) = f^eq_i(x + xi_i)) so that the first pull yields f^eq(x).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <type_traits>

#include "lbm.h"
#include "lbm_cell.hpp"
#include "lbm_internal.hpp"
#include "lbm_step2.hpp"
#include "lbm_step3.hpp"

using namespace lbm;

namespace lbm {

thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    return set_error(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace lbm

// Reduction scratch of lbm_moments_noalloc: 5 per-block partial sums for up to
// kNoAllocMaxBlocks blocks of the per-cell launch, then 5 totals.  One copy per device, held
// until the process ends.  In host code `scratch` is only a symbol: its device address comes
// from hipGetSymbolAddress (per device, at context creation) and is kept in lbm_ctx.
constexpr int kNoAllocMaxBlocks = 65536;
static __device__ __align__(256) double scratch[5 * kNoAllocMaxBlocks + 8];

namespace lbm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
int scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(LBM_EUNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc != LBM_OK) return rc;
        g_scratch_addr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[device];
    return LBM_OK;
}

}  // namespace

Launch launch_for(int nx, int ny) {
    int bw = 256;
    while (bw > 64 && bw / 2 >= nx) bw /= 2;
    const int bh = 256 / bw;
    Launch l;
    l.block = dim3(bw, bh, 1);
    l.grid = dim3((nx + bw - 1) / bw, (ny + bh - 1) / bh, 1);
    return l;
}

StepShape step_shape(int nx, int ny, int rows, int xcd) {
    const Launch l = launch_for(nx, ny);
    StepShape sh;
    sh.bw = (int)l.block.x;
    sh.bh = (int)l.block.y;
    sh.rows = rows;
    sh.xcd = xcd;
    sh.gx = l.grid.x;
    sh.gy = (unsigned)((ny + sh.bh * rows - 1) / (sh.bh * rows));
    return sh;
}

// Planes are padded by a further 1 KiB so that the nine (eighteen) concurrent streams of a step
// do not sit at power-of-two distances, which on MI355X costs 1-2% of bandwidth on square
// power-of-two grids (they then map onto the same HBM channels at the same time).
#ifndef LBM_PLANE_SKEW_BYTES
#define LBM_PLANE_SKEW_BYTES 1024
#endif

long long plane_elems(int nx, int ny, int prec) {
    const long long align = 256 / elem_size(prec);
    const long long n = (long long)nx * ny;
    return (n + align - 1) / align * align + LBM_PLANE_SKEW_BYTES / elem_size(prec);
}

int validate_omega(const double* w) {
    if (!w) return set_error(LBM_EINVAL, "omega is NULL");
    for (int k = 0; k < LBM_NOMEGA; ++k)
        if (!(w[k] >= 0.0 && w[k] <= 2.0))
            return set_error(LBM_EINVAL, "omega[%d] = %g outside [0, 2]", k, w[k]);
    return LBM_OK;
}

int validate_model(int model, int eq_order) {
    switch (model) {
        case LBM_BGK: case LBM_RM: case LBM_HM: case LBM_PR: case LBM_RR: case LBM_STREAM_ONLY:
            return LBM_OK;
        case LBM_CM: case LBM_CHM: case LBM_K:
            if (eq_order != 4)
                return set_error(LBM_EUNSUPPORTED,
                                 "model %d relaxes central quantities and needs eq_order 4 (got %d)",
                                 model, eq_order);
            return LBM_OK;
        default:
            return set_error(LBM_EINVAL, "unknown model %d", model);
    }
}

}  // namespace lbm

namespace {

// ---------------------------------------------------------------------------------------------
// kernels

template <int MODEL, int PREC, int ROWS>
__global__ __launch_bounds__(256) void k_step(const typename Store<PREC>::S* __restrict__ src,
                                              typename Store<PREC>::S* __restrict__ dst, Geom g,
                                              Coef<typename Store<PREC>::R> c,
                                              Ref<typename Store<PREC>::R> ref, int N, int step,
                                              int* __restrict__ blowup, unsigned gx, unsigned nb,
                                              int xcd) {
    using R = typename Store<PREC>::R;
    unsigned bx, by;
    tile_of_block(blockIdx.x, gx, nb, xcd, bx, by);
    const int x = bx * blockDim.x + threadIdx.x;
    const int y0 = by * blockDim.y * ROWS + threadIdx.y;
    if (x >= g.nx) return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + r * (int)blockDim.y;
        if (y < g.ny) {
            const Nbr nb4 = neighbours(x, y, g.nx, g.ny);
            R h[9];
            pull_load(src, g.plane, nb4, h);
            double rho_d;
            const Macro<R> m = macro_of<typename Store<PREC>::S>(h, ref, rho_d);
            flag_bad(!(rho_d > 0.0), blowup, step);
            collide<MODEL>(h, m, ref, c, N);
            store_cell(dst, g.plane, nb4.r0 + (unsigned)x, h);
        }
    }
}


// Strip height a new context starts with (ring of 8 rows), 0 for single steps.  Measured on
// MI355X (CM, double shear layer): two steps per launch win in FP32 and FP64 from 512^2 up
// (strips of 16 rows: 256 blocks at 512^2), and in FP16, whose step is bound by arithmetic
// rather than bytes, only once strips of 40 rows still give 1024 blocks (2048^2 and up); FP64
// takes strips of 64 rows when they give 1024 blocks.  (At 4096^2 FP16 runs 1-5% faster on
// 40-row strips than on 32 or 64: strip starts a power-of-two number of rows apart put the
// concurrently running strips at addresses a large power of two apart.)
int default_fusion_strip(int nx, int ny, int prec) {
    const long long sx = (nx + kStripW - 1) / kStripW;
    const long long s16 = sx * ((ny + 15) / 16), s40 = sx * ((ny + 39) / 40), s64 = sx * ((ny + 63) / 64);
    if (prec == LBM_F16_SHIFTED) return s40 >= 1024 ? 40 : 0;
    if (prec == LBM_F64 && s64 >= 1024) return 64;
    return s16 >= 256 ? 16 : 0;
}

// Strip width of the two-step kernel for a model and precision.  Measured at 4096^2: in FP32 every
// model gains from strips of 128 columns (two waves per row: half the edge lines and halo nodes
// per column), 2-5% over 64 columns; FP64 (bandwidth-bound on 64-row strips) and FP16 (bound by
// arithmetic) do not, and keep 64.
constexpr bool wide_strips(int /*model*/, int prec) { return prec == LBM_F32_SHIFTED; }

// (ring rows, strip rows) a new context starts with on 128-column strips, measured at 4096^2 in
// FP32: a ring of 4 rows on 20-row strips for every model but BGK, whose light collision gains
// most from one pass of a ring of 8 rows per 8-row strip (1-2% over 16-row strips, which start a
// power of two apart; see default_fusion_strip).
struct FusionPick {
    int ring, strip;
};
constexpr FusionPick wide_default(int model) { return model == LBM_BGK ? FusionPick{8, 8} : FusionPick{4, 20}; }

// Three steps per launch for a new FP32 or FP64 context while its 64-column strips number at least
// kDeepMinStrips.  The strip height is about gsx ny / sqrt(nx ny) rows (n / 64 on an n x n grid: as
// many strips as columns), a multiple of 8 in [8, 64], and 128 in place of 64 (deep_pick has the
// ring and the final height).  Three steps against two per launch, first measured on MI355X with a
// ring of 4 rows (double shear layer, BGK / K): FP32 512^2 77 / 66k MLUPS against 59 / 54k, 1024^2
// 129 / 118k against 97 / 91k, 2048^2 161 / 146k against 118 / 117k, 4096^2 186 / 169k against
// 145 / 138k; FP64 2048^2 75 / 72k against 61 / 62k, 4096^2 86 / 83k against 75 / 74k.
constexpr long long kDeepMinStrips = 512;

int deep_strip(int nx, int ny, int prec) {
    const double gsx = (double)((nx + kStripW - 1) / kStripW);
    const int h = 8 * (int)(gsx * ny / std::sqrt((double)nx * ny) / 8.0 + 0.5);
    const int hs = h < 8 ? 8 : (h > 64 ? 64 : h);
    return (prec == LBM_F32_SHIFTED && hs == 64) ? 128 : hs;
}

// Ring and strip height of a model's three-step launches on a new context (deep_strip's count of
// 64-column strips is at least kDeepMinStrips).  Measured on MI355X (double shear layer, MLUPS):
// - FP32: a ring of 8 rows (8 waves, 48 KiB of LDS, three workgroups per CU) for every model, at
//   4096^2 with 80-row strips 174-191k against 170-185k with a ring of 4 (K / BGK); with the strips
//   dealt to the XCDs by column groups, 128-row strips (where deep_strip reaches 64) run another
//   1-2.5% faster than 80 (96, 112 and 160-256 rows slower) and are the default; at 2048^2 152 /
//   166k against 145 / 160k, at 512^2 78 / 91k against 67 / 78k.  Where the strip count lies just
//   above one round of workgroups (three per CU), up to 1.5 rounds, the strips are made taller until
//   they fit one round: at 1024^2, 24-row strips 118 / 131k against 106 / 120k with 16 rows (a ring
//   of 4 rows on 16-row strips: 118 / 129k).
// - FP64: a ring of 8 rows on 48-column strips (74 KiB, two workgroups of 8 waves per CU) for every
//   model, 128 rows where deep_strip gives 64: at 4096^2 with the strips dealt to the XCDs by column
//   groups BGK 98k, RM 98k, K 91k, PR 103k (ring of 4 rows on 64-row strips: 98k, 91k, 84k, 96k;
//   in bands of strip rows, 96-row strips: 95k, 97k, 90k, 100k).
FusionPick deep_pick(int model, int nx, int ny, int prec, int cus) {
    const int hs = deep_strip(nx, ny, prec);
    if (prec == LBM_F64) return FusionPick{8, hs == 64 ? 128 : hs};
    const long long gsx = (nx + kStripW - 1) / kStripW;
    const long long round = 3LL * cus;
    int h = hs;
    auto strips = [&](int r) { return gsx * ((ny + r - 1) / r); };
    if (cus > 0 && strips(h) > round && 2 * strips(h) <= 3 * round)
        while (strips(h) > round && h < 256) h += 8;
    return FusionPick{8, h};
}

// Widest strip for a model and precision; the launch uses it only while it still gives at least
// kWideMinStrips strips (otherwise 64 columns keep enough workgroups in flight on small grids).
constexpr long long kWideMinStrips = 1024;

template <int MODEL, int PREC>
constexpr int strip_width() {
    return wide_strips(MODEL, PREC == kF32 ? LBM_F32_SHIFTED : (PREC == kF64 ? LBM_F64 : LBM_F16_SHIFTED))
               ? 2 * kStripW
               : kStripW;
}

template <int MODEL, int PREC, int RING, int W, bool MID = false>
__global__ __launch_bounds__(256) void k_step2(const typename Store<PREC>::S* __restrict__ src,
                                               typename Store<PREC>::S* __restrict__ dst, Geom g,
                                               Coef<typename Store<PREC>::R> c,
                                               Ref<typename Store<PREC>::R> ref, int N, int step,
                                               int* __restrict__ blowup, unsigned gsx, int hs,
                                               typename Store<PREC>::S* __restrict__ mid) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    __shared__ S ring[9][RING + 2][W + 2];
    // FP16 (64-column strips, one 128-byte line per plane and row): strips dealt to the XCDs by
    // groups of 8 strip columns, so neighbouring strips share their edge lines in one L2 (bands of
    // whole strip rows: +2-7% over the hardware order; column groups of 8 another 1-4%, of 16
    // 0-2%); FP32 (128 columns) and FP64 measured 2-6% slower in bands and within 3% either way in
    // column groups, and keep the hardware order
    unsigned sx, sy;
    if constexpr (PREC == kF16)
        strip_of_block_grouped(blockIdx.x, gsx, gridDim.x, 8, sx, sy);
    else
        tile_of_block(blockIdx.x, gsx, gridDim.x, 0, sx, sy);
    const int x0 = (int)sx * W;
    const int ys = (int)sy * hs;
    strip_two_steps<RING, W, false, true, MID>(
        ring, src, dst, g, ref, x0, ys, min(ys + hs, g.ny), step, blowup,
        [&](R(&h)[9], const Macro<R>& m) { collide<MODEL>(h, m, ref, c, N); }, mid);
}

// Three steps per launch: strips of W columns and hs rows, two LDS rings (strip_three_steps).
// A ring of 8 rows runs 8 waves (512 threads), one row each per pass: the two halo passes then cost
// two wave-collisions per 24 useful ones instead of per 12 with a ring of 4 rows.
template <int RING> constexpr int step3_waves() { return RING == 8 ? 8 : 4; }

template <int MODEL, int PREC, int RING, int W>
__global__ __launch_bounds__(64 * step3_waves<RING>()) void k_step3(const typename Store<PREC>::S* __restrict__ src,
                                               typename Store<PREC>::S* __restrict__ dst, Geom g,
                                               Coef<typename Store<PREC>::R> c,
                                               Ref<typename Store<PREC>::R> ref, int N, int step,
                                               int* __restrict__ blowup, unsigned gsx, int hs) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    __shared__ S ring1[9][RING + 2][W + 4];
    __shared__ S ring2[9][RING + 2][W + 2];
    // FP32: strips dealt to the XCDs by groups of 16 strip columns, so that neighbouring strips
    // share their edge lines in one L2 (in hardware order the traffic was 1.57x the algorithmic
    // bytes; bands of whole strip rows: 1.05x and 2-3% faster; column groups of 16 another 1-4%
    // over bands, groups of 8 and 32 slightly less); FP64 on 64-column strips (not a default: FP64
    // takes the 48-column k_step3n) measured 2% slower in bands and keeps the hardware order
    unsigned sx, sy;
    if constexpr (PREC == kF32)
        strip_of_block_grouped(blockIdx.x, gsx, gridDim.x, 16, sx, sy);
    else
        tile_of_block(blockIdx.x, gsx, gridDim.x, 0, sx, sy);
    const int x0 = (int)sx * W;
    const int ys = (int)sy * hs;
    strip_three_steps<RING, W, false, true, step3_waves<RING>()>(
        ring1, ring2, src, dst, g, ref, x0, ys, min(ys + hs, g.ny), step, blowup,
        [&](R(&h)[9], const Macro<R>& m) { collide<MODEL>(h, m, ref, c, N); });
}

// Three steps per launch on strips of WP columns whose halo columns fit the wave (FP64: WP = 48;
// measured at 4096^2 against 64-column strips: BGK 96 against 86k MLUPS, K 82 against 80k).
template <int MODEL, int PREC, int RING, int WP>
__global__ __launch_bounds__(64 * step3_waves<RING>()) void k_step3n(const typename Store<PREC>::S* __restrict__ src,
                                                typename Store<PREC>::S* __restrict__ dst, Geom g,
                                                Coef<typename Store<PREC>::R> c,
                                                Ref<typename Store<PREC>::R> ref, int N, int step,
                                                int* __restrict__ blowup, unsigned gsx, int hs) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    __shared__ S ring1[9][RING + 2][WP + 4];
    __shared__ S ring2[9][RING + 2][WP + 3];
    // strips dealt to the XCDs by groups of 16 strip columns (bands of whole strip rows measured 1-4%
    // faster than the hardware order; column groups with 128-row strips another 1-3%, and less
    // sensitive to the strip height)
    unsigned sx, sy;
    strip_of_block_grouped(blockIdx.x, gsx, gridDim.x, 16, sx, sy);
    const int x0 = (int)sx * WP;
    const int ys = (int)sy * hs;
    strip_three_steps_narrow<RING, WP, false, true, step3_waves<RING>()>(
        ring1, ring2, src, dst, g, ref, x0, ys, min(ys + hs, g.ny), step, blowup,
        [&](R(&h)[9], const Macro<R>& m) { collide<MODEL>(h, m, ref, c, N); });
}

// Macroscopic fields of the state f(., n) (pulled from the post-collision copy) and per-block
// partial sums of {rho, rho ux, rho uy, rho |u|^2 / 2, |u|^2} in FP64.
template <int PREC>
__global__ __launch_bounds__(256) void k_moments(const typename Store<PREC>::S* __restrict__ src,
                                                 Geom g, Ref<double> ref, double* __restrict__ rho,
                                                 double* __restrict__ ux, double* __restrict__ uy,
                                                 double* __restrict__ partials, int step,
                                                 int* __restrict__ blowup) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < g.nx && y < g.ny) {
        const Nbr nb = neighbours(x, y, g.nx, g.ny);
        double h[9];
        pull_load(src, g.plane, nb, h);
        double r = ref.rho + (((h[0] + (h[1] + h[3])) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8])));
        const double jx = ((h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7])) + ref.rho * ref.ux;
        const double jy = ((h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8])) + ref.rho * ref.uy;
        const double u = jx / r, w = jy / r;
        const unsigned c = nb.r0 + (unsigned)x;
        if (rho) rho[c] = r;
        if (ux) ux[c] = u;
        if (uy) uy[c] = w;
        const double u2 = u * u + w * w;
        v[0] = r; v[1] = r * u; v[2] = r * w; v[3] = 0.5 * r * u2; v[4] = u2;
        flag_bad(!(r > 0.0), blowup, step);
    }
    block_sum<5>(v, partials + 5 * (size_t)(blockIdx.y * gridDim.x + blockIdx.x));
}

// Sum nblocks rows of 5 partials in a fixed order (one block of 256 threads).
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int nblocks,
                                                  double* __restrict__ out) {
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < 5; ++k) v[k] += partials[5 * (size_t)b + k];
    block_sum<5>(v, out);
}

// The six totals of lbm_moments from the five reduced sums, written to device memory
// (the mean of |u|^2 divided by the node count, and the step), one thread.
__global__ void k_totals_out(const double* __restrict__ t, double nodes, double step, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int k = 0; k < 4; ++k) out[k] = t[k];
        out[4] = t[4] / nodes;
        out[5] = step;
    }
}

// Unshifted FP64 pre-collision populations, [q][y][x] dense.
template <int PREC>
__global__ __launch_bounds__(256) void k_get_state(const typename Store<PREC>::S* __restrict__ src,
                                                   Geom g, Pop9 fref, double* __restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const Nbr nb = neighbours(x, y, g.nx, g.ny);
    double h[9];
    pull_load(src, g.plane, nb, h);
    const size_t cells = (size_t)g.nx * g.ny, c = nb.r0 + (size_t)x;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i * cells + c] = h[i] + fref.v[i];
}

// Store pre-collision populations f (unshifted FP64, [q][y][x]) pre-streamed backwards so that
// the next pull returns f(x): value i of node x goes to node x - xi_i.
template <int PREC>
__global__ __launch_bounds__(256) void k_set_state(typename Store<PREC>::S* __restrict__ dst,
                                                   Geom g, Pop9 fref,
                                                   const double* __restrict__ f) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const size_t cells = (size_t)g.nx * g.ny, c = (size_t)y * g.nx + x;
    double h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = f[i * cells + c] - fref.v[i];
    prestream_store(dst, g, x, y, h);
}

// f(., 0) = f^eq_N(rho, u), stored pre-streamed like k_set_state.  FP64 arithmetic.
template <int PREC>
__global__ __launch_bounds__(256) void k_init_eq(typename Store<PREC>::S* __restrict__ dst, Geom g,
                                                 Ref<double> ref, int N, const double* __restrict__ rho,
                                                 const double* __restrict__ ux,
                                                 const double* __restrict__ uy) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const size_t c = (size_t)y * g.nx + x;
    double h[9];
    eq_deviation(rho[c], ux[c], uy[c], ref, N, h);
    prestream_store(dst, g, x, y, h);
}

// ---------------------------------------------------------------------------------------------
// host side

template <int MODEL, int PREC, int ROWS>
void launch_step_r(lbm_ctx* ctx, const StepShape& sh, const Coef<typename Store<PREC>::R>& c,
                   int src_copy) {
    using S = typename Store<PREC>::S;
    const S* src = reinterpret_cast<const S*>(ctx->copy(src_copy));
    S* dst = reinterpret_cast<S*>(ctx->copy(src_copy ^ 1));
    const unsigned nb = sh.gx * sh.gy;
    hipLaunchKernelGGL((k_step<MODEL, PREC, ROWS>), dim3(nb), dim3(sh.bw, sh.bh), 0, ctx->stream,
                       src, dst, ctx->geom(), c, ref_as<typename Store<PREC>::R>(ctx->ref),
                       ctx->eq_order, (int)ctx->step, ctx->d_flag, sh.gx, nb, sh.xcd);
}

template <int MODEL, int PREC, int ROWS>
void launch_step_raw_r(lbm_ctx* ctx, const StepShape& sh, const Coef<typename Store<PREC>::R>& c,
                       const void* src, void* dst, int step) {
    using S = typename Store<PREC>::S;
    const unsigned nb = sh.gx * sh.gy;
    hipLaunchKernelGGL((k_step<MODEL, PREC, ROWS>), dim3(nb), dim3(sh.bw, sh.bh), 0, ctx->stream,
                       reinterpret_cast<const S*>(src), reinterpret_cast<S*>(dst), ctx->geom(), c,
                       ref_as<typename Store<PREC>::R>(ctx->ref), ctx->eq_order, step,
                       ctx->d_flag, sh.gx, nb, sh.xcd);
}

template <int MODEL, int PREC>
void launch_step_raw_t(lbm_ctx* ctx, const StepShape& sh, const Coef<typename Store<PREC>::R>& c,
                       const void* src, void* dst, int step) {
    switch (sh.rows) {
        case 4: launch_step_raw_r<MODEL, PREC, 4>(ctx, sh, c, src, dst, step); break;
        case 2: launch_step_raw_r<MODEL, PREC, 2>(ctx, sh, c, src, dst, step); break;
        default: launch_step_raw_r<MODEL, PREC, 1>(ctx, sh, c, src, dst, step); break;
    }
}

template <int PREC>
void launch_step_raw_p(lbm_ctx* ctx, int model, const double* w, const StepShape& sh, const void* src,
                       void* dst, int step) {
    const Coef<typename Store<PREC>::R> c = make_coef<typename Store<PREC>::R>(w);
    switch (model) {
        case LBM_BGK: launch_step_raw_t<kBGK, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_RM: launch_step_raw_t<kRM, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_HM: launch_step_raw_t<kHM, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_CM: launch_step_raw_t<kCM, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_CHM: launch_step_raw_t<kCHM, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_K: launch_step_raw_t<kK, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_PR: launch_step_raw_t<kPR, PREC>(ctx, sh, c, src, dst, step); break;
        case LBM_RR: launch_step_raw_t<kRR, PREC>(ctx, sh, c, src, dst, step); break;
        default: launch_step_raw_t<kStreamOnly, PREC>(ctx, sh, c, src, dst, step); break;
    }
}

// One launch of k_step2 with strips of W columns.
template <int MODEL, int PREC, int RING, int W, bool MID>
void launch_step2_w(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, const void* src, void* mid,
                    void* dst, int step) {
    using S = typename Store<PREC>::S;
    const unsigned gsx = (unsigned)((ctx->nx + W - 1) / W);
    const unsigned gsy = (unsigned)((ctx->ny + hs - 1) / hs);
    hipLaunchKernelGGL((k_step2<MODEL, PREC, RING, W, MID>), dim3(gsx * gsy), dim3(256), 0, ctx->stream,
                       reinterpret_cast<const S*>(src), reinterpret_cast<S*>(dst), ctx->geom(), c,
                       ref_as<typename Store<PREC>::R>(ctx->ref), ctx->eq_order, step, ctx->d_flag, gsx, hs,
                       reinterpret_cast<S*>(mid));
}

// The model's widest strips while they give kWideMinStrips strips, else 64 columns.
template <int MODEL, int PREC, int RING, bool MID>
void launch_step2_any(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, const void* src, void* mid,
                      void* dst, int step) {
    constexpr int WW = strip_width<MODEL, PREC>();
    if constexpr (WW != kStripW) {
        const long long strips = (long long)((ctx->nx + WW - 1) / WW) * ((ctx->ny + hs - 1) / hs);
        if (strips >= kWideMinStrips) {
            launch_step2_w<MODEL, PREC, RING, WW, MID>(ctx, c, hs, src, mid, dst, step);
            return;
        }
    }
    launch_step2_w<MODEL, PREC, RING, kStripW, MID>(ctx, c, hs, src, mid, dst, step);
}

template <int MODEL, int PREC, int RING>
void launch_step2_r(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, int src_copy) {
    launch_step2_any<MODEL, PREC, RING, false>(ctx, c, hs, ctx->copy(src_copy), nullptr, ctx->copy(src_copy ^ 1),
                                               (int)ctx->step);
}

// Two raw steps src -> dst (ring of 8 rows, strips of hs rows); with mid != NULL the state after
// the first step is also written there.
template <int MODEL, int PREC>
void launch_step2_raw_t(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, const void* src, void* mid,
                        void* dst, int step) {
    if (mid)
        launch_step2_any<MODEL, PREC, 8, true>(ctx, c, hs, src, mid, dst, step);
    else
        launch_step2_any<MODEL, PREC, 8, false>(ctx, c, hs, src, nullptr, dst, step);
}

template <int PREC>
void launch_step2_raw_p(lbm_ctx* ctx, int model, const double* w, int hs, const void* src, void* mid, void* dst,
                        int step) {
    const Coef<typename Store<PREC>::R> c = make_coef<typename Store<PREC>::R>(w);
    switch (model) {
        case LBM_BGK: launch_step2_raw_t<kBGK, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_RM: launch_step2_raw_t<kRM, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_HM: launch_step2_raw_t<kHM, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_CM: launch_step2_raw_t<kCM, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_CHM: launch_step2_raw_t<kCHM, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_K: launch_step2_raw_t<kK, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_PR: launch_step2_raw_t<kPR, PREC>(ctx, c, hs, src, mid, dst, step); break;
        case LBM_RR: launch_step2_raw_t<kRR, PREC>(ctx, c, hs, src, mid, dst, step); break;
        default: launch_step2_raw_t<kStreamOnly, PREC>(ctx, c, hs, src, mid, dst, step); break;
    }
}

template <int MODEL, int PREC>
void launch_step2_t(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int ring, int hs, int src_copy) {
    switch (ring) {
        case 4: launch_step2_r<MODEL, PREC, 4>(ctx, c, hs, src_copy); break;
        case 16:
            // the ring must fit in the 160 KiB of LDS a workgroup can have
            if constexpr (9 * 18 * (strip_width<MODEL, PREC>() + 2) * sizeof(typename Store<PREC>::S) <= 160 * 1024)
                launch_step2_r<MODEL, PREC, 16>(ctx, c, hs, src_copy);
            else
                launch_step2_r<MODEL, PREC, 8>(ctx, c, hs, src_copy);
            break;
        default: launch_step2_r<MODEL, PREC, 8>(ctx, c, hs, src_copy); break;
    }
}

template <int PREC>
void launch_step2_p(lbm_ctx* ctx, int model, const double* w, int ring, int hs, int src_copy) {
    const Coef<typename Store<PREC>::R> c = make_coef<typename Store<PREC>::R>(w);
    switch (model) {
        case LBM_BGK: launch_step2_t<kBGK, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_RM: launch_step2_t<kRM, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_HM: launch_step2_t<kHM, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_CM: launch_step2_t<kCM, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_CHM: launch_step2_t<kCHM, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_K: launch_step2_t<kK, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_PR: launch_step2_t<kPR, PREC>(ctx, c, ring, hs, src_copy); break;
        case LBM_RR: launch_step2_t<kRR, PREC>(ctx, c, ring, hs, src_copy); break;
        default: launch_step2_t<kStreamOnly, PREC>(ctx, c, ring, hs, src_copy); break;
    }
}

// One launch of k_step3 (three steps, steps step .. step + 2) with strips of W columns from the
// state src to dst.
template <int MODEL, int PREC, int RING, int W>
void launch_step3_w(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, const void* src, void* dst,
                    int step) {
    using S = typename Store<PREC>::S;
    const unsigned gsx = (unsigned)((ctx->nx + W - 1) / W);
    const unsigned gsy = (unsigned)((ctx->ny + hs - 1) / hs);
    hipLaunchKernelGGL((k_step3<MODEL, PREC, RING, W>), dim3(gsx * gsy), dim3(64 * step3_waves<RING>()), 0, ctx->stream,
                       reinterpret_cast<const S*>(src), reinterpret_cast<S*>(dst), ctx->geom(), c,
                       ref_as<typename Store<PREC>::R>(ctx->ref), ctx->eq_order, step, ctx->d_flag, gsx, hs);
}

// FP64 three-step strips: 48 columns, the halo columns inside the wave (no halo passes), each row
// segment three whole 128-byte lines; the rings take 74 KiB with a ring of 8 rows (two workgroups of
// 8 waves per CU, the default) and 44 KiB with 4 (three workgroups of 4 waves).
constexpr int kNarrowW = 48;

// One launch of k_step3n (FP64 narrow strips) from the state src to dst.
template <int MODEL, int PREC, int RING, int WP>
void launch_step3n_w(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int hs, const void* src, void* dst,
                     int step) {
    using S = typename Store<PREC>::S;
    const unsigned gsx = (unsigned)((ctx->nx + WP - 1) / WP);
    const unsigned gsy = (unsigned)((ctx->ny + hs - 1) / hs);
    hipLaunchKernelGGL((k_step3n<MODEL, PREC, RING, WP>), dim3(gsx * gsy), dim3(64 * step3_waves<RING>()), 0, ctx->stream,
                       reinterpret_cast<const S*>(src), reinterpret_cast<S*>(dst), ctx->geom(), c,
                       ref_as<typename Store<PREC>::R>(ctx->ref), ctx->eq_order, step, ctx->d_flag, gsx, hs);
}

// Three steps per launch: FP32 on 64-column strips (the two rings of 128-column strips take 56 KiB
// of LDS with a ring of 4 rows, two workgroups per CU, and measured 10-25% slower), FP64 on 48-column
// narrow strips with either ring.
template <int MODEL, int PREC>
void launch_step3_t(lbm_ctx* ctx, const Coef<typename Store<PREC>::R>& c, int ring, int hs, const void* src,
                    void* dst, int step) {
    if constexpr (PREC == kF64) {
        if (ring == 4)
            launch_step3n_w<MODEL, PREC, 4, kNarrowW>(ctx, c, hs, src, dst, step);
        else
            launch_step3n_w<MODEL, PREC, 8, kNarrowW>(ctx, c, hs, src, dst, step);
    } else if constexpr (PREC == kF32) {
        if (ring == 4)
            launch_step3_w<MODEL, PREC, 4, kStripW>(ctx, c, hs, src, dst, step);
        else
            launch_step3_w<MODEL, PREC, 8, kStripW>(ctx, c, hs, src, dst, step);
    }
}

template <int PREC>
void launch_step3_p(lbm_ctx* ctx, int model, const double* w, int ring, int hs, const void* src, void* dst,
                    int step) {
    const Coef<typename Store<PREC>::R> c = make_coef<typename Store<PREC>::R>(w);
    switch (model) {
        case LBM_BGK: launch_step3_t<kBGK, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_RM: launch_step3_t<kRM, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_HM: launch_step3_t<kHM, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_CM: launch_step3_t<kCM, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_CHM: launch_step3_t<kCHM, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_K: launch_step3_t<kK, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_PR: launch_step3_t<kPR, PREC>(ctx, c, ring, hs, src, dst, step); break;
        case LBM_RR: launch_step3_t<kRR, PREC>(ctx, c, ring, hs, src, dst, step); break;
        default: launch_step3_t<kStreamOnly, PREC>(ctx, c, ring, hs, src, dst, step); break;
    }
}

template <int MODEL, int PREC>
void launch_step_t(lbm_ctx* ctx, const StepShape& sh, const Coef<typename Store<PREC>::R>& c,
                   int src_copy) {
    switch (sh.rows) {
        case 4: launch_step_r<MODEL, PREC, 4>(ctx, sh, c, src_copy); break;
        case 2: launch_step_r<MODEL, PREC, 2>(ctx, sh, c, src_copy); break;
        default: launch_step_r<MODEL, PREC, 1>(ctx, sh, c, src_copy); break;
    }
}

template <int PREC>
void launch_step_p(lbm_ctx* ctx, int model, const double* w, const StepShape& sh, int src_copy) {
    const Coef<typename Store<PREC>::R> c = make_coef<typename Store<PREC>::R>(w);
    switch (model) {
        case LBM_BGK: launch_step_t<kBGK, PREC>(ctx, sh, c, src_copy); break;
        case LBM_RM: launch_step_t<kRM, PREC>(ctx, sh, c, src_copy); break;
        case LBM_HM: launch_step_t<kHM, PREC>(ctx, sh, c, src_copy); break;
        case LBM_CM: launch_step_t<kCM, PREC>(ctx, sh, c, src_copy); break;
        case LBM_CHM: launch_step_t<kCHM, PREC>(ctx, sh, c, src_copy); break;
        case LBM_K: launch_step_t<kK, PREC>(ctx, sh, c, src_copy); break;
        case LBM_PR: launch_step_t<kPR, PREC>(ctx, sh, c, src_copy); break;
        case LBM_RR: launch_step_t<kRR, PREC>(ctx, sh, c, src_copy); break;
        default: launch_step_t<kStreamOnly, PREC>(ctx, sh, c, src_copy); break;
    }
}

template <int PREC>
void launch_moments_p(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* partials) {
    using S = typename Store<PREC>::S;
    const Launch l = launch_for(ctx->nx, ctx->ny);
    hipLaunchKernelGGL((k_moments<PREC>), l.grid, l.block, 0, ctx->stream,
                       reinterpret_cast<const S*>(ctx->copy(ctx->cur)), ctx->geom(), ctx->ref, rho,
                       ux, uy, partials, (int)ctx->step, ctx->d_flag);
}

template <int PREC>
void launch_get_p(lbm_ctx* ctx, double* f) {
    using S = typename Store<PREC>::S;
    const Launch l = launch_for(ctx->nx, ctx->ny);
    hipLaunchKernelGGL((k_get_state<PREC>), l.grid, l.block, 0, ctx->stream,
                       reinterpret_cast<const S*>(ctx->copy(ctx->cur)), ctx->geom(), ctx->fref, f);
}

template <int PREC>
void launch_set_p(lbm_ctx* ctx, const double* f) {
    using S = typename Store<PREC>::S;
    const Launch l = launch_for(ctx->nx, ctx->ny);
    hipLaunchKernelGGL((k_set_state<PREC>), l.grid, l.block, 0, ctx->stream,
                       reinterpret_cast<S*>(ctx->copy(ctx->cur)), ctx->geom(), ctx->fref, f);
}

template <int PREC>
void launch_init_p(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy) {
    using S = typename Store<PREC>::S;
    const Launch l = launch_for(ctx->nx, ctx->ny);
    hipLaunchKernelGGL((k_init_eq<PREC>), l.grid, l.block, 0, ctx->stream,
                       reinterpret_cast<S*>(ctx->copy(ctx->cur)), ctx->geom(), ctx->ref,
                       ctx->eq_order, rho, ux, uy);
}

#define LBM_DISPATCH_PREC(prec, fn, ...)                      \
    do {                                                      \
        switch (prec) {                                       \
            case LBM_F64: fn<kF64>(__VA_ARGS__); break;       \
            case LBM_F32_SHIFTED: fn<kF32>(__VA_ARGS__); break; \
            default: fn<kF16>(__VA_ARGS__); break;            \
        }                                                     \
    } while (0)

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int reset_flag(lbm_ctx* ctx) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, ctx->d_flag, 1, INT_MAX);
    return check_hip(hipGetLastError(), "reset blow-up flag");
}

}  // namespace

namespace lbm {

int reset_blowup(lbm_ctx* ctx) { return reset_flag(ctx); }

int reduce_partials(lbm_ctx* ctx) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->nblocks, ctx->d_tot);
    return check_hip(hipGetLastError(), "finalize kernel launch");
}

}  // namespace lbm

// -------------------------------------------------------------------------------------------------
// C ABI

extern "C" {

size_t lbm_population_bytes(int nx, int ny, int prec) {
    if (nx < 2 || ny < 2 || prec < LBM_F64 || prec > LBM_F16_SHIFTED) return 0;
    if ((long long)nx * ny * 9 >= (1LL << 31)) return 0;
    return (size_t)(2 * 9 * plane_elems(nx, ny, prec) * elem_size(prec));
}

int lbm_init(lbm_ctx** out, int nx, int ny, int prec, int eq_order, double rho0, const double* rho,
             const double* ux, const double* uy, void* pop_buf, size_t pop_bytes,
             void* hip_stream) {
    return lbm_init_shifted(out, nx, ny, prec, eq_order, rho0, 0.0, 0.0, rho, ux, uy, pop_buf,
                            pop_bytes, hip_stream);
}

int lbm_init_shifted(lbm_ctx** out, int nx, int ny, int prec, int eq_order, double rho0,
                     double ux0, double uy0, const double* rho, const double* ux,
                     const double* uy, void* pop_buf, size_t pop_bytes, void* hip_stream) {
    if (!out) return set_error(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 2 || ny < 2) return set_error(LBM_EINVAL, "grid %d x %d: each side must be >= 2", nx, ny);
    if ((long long)nx * ny * 9 >= (1LL << 31))
        return set_error(LBM_EINVAL, "grid %d x %d too large (9 nx ny must be < 2^31)", nx, ny);
    if (prec < LBM_F64 || prec > LBM_F16_SHIFTED) return set_error(LBM_EINVAL, "unknown precision %d", prec);
    if (eq_order < 2 || eq_order > 4) return set_error(LBM_EINVAL, "eq_order %d not in {2,3,4}", eq_order);
    if (prec != LBM_F64 && !(rho0 > 0.0)) return set_error(LBM_EINVAL, "rho0 must be > 0 (got %g)", rho0);
    if (prec != LBM_F64 && !(ux0 * ux0 + uy0 * uy0 < 1.0))
        return set_error(LBM_EINVAL, "reference velocity (%g, %g) must have |U| < 1", ux0, uy0);
    if (!rho || !ux || !uy) return set_error(LBM_EINVAL, "rho/ux/uy must be device pointers");
    if (!pop_buf) return set_error(LBM_EINVAL, "pop_buf is NULL");
    if (reinterpret_cast<uintptr_t>(pop_buf) % 256 != 0)
        return set_error(LBM_EINVAL, "pop_buf must be 256-byte aligned");
    const size_t need = lbm_population_bytes(nx, ny, prec);
    if (pop_bytes < need)
        return set_error(LBM_EINVAL, "pop_bytes %zu < required %zu", pop_bytes, need);

    lbm_ctx* ctx = new lbm_ctx();
    ctx->nx = nx;
    ctx->ny = ny;
    ctx->prec = prec;
    ctx->eq_order = eq_order;
    ctx->ref = storage_reference(prec, rho0, ux0, uy0);
    ctx->fref = reference_populations(ctx->ref, eq_order);
    ctx->buf = static_cast<char*>(pop_buf);
    ctx->bytes = pop_bytes;
    ctx->plane = plane_elems(nx, ny, prec);
    ctx->esize = elem_size(prec);
    ctx->cur = 0;
    ctx->step = 0;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    const Launch l = launch_for(nx, ny);
    ctx->nblocks = (int)(l.grid.x * l.grid.y);
    // FP16 rows are 128 bytes per wave and plane: two nodes per thread keep enough bytes in
    // flight (measured on MI355X; lbm_autotune can revise it)
    for (int k = 0; k < 9; ++k) ctx->rows[k] = prec == LBM_F16_SHIFTED ? 2 : 1;
    const int fstrip = default_fusion_strip(nx, ny, prec);
    const int dstrip = deep_strip(nx, ny, prec);
    const bool deep = prec != LBM_F16_SHIFTED && nx >= 2 && ny >= 2 &&
                      (long long)((nx + kStripW - 1) / kStripW) * ((ny + dstrip - 1) / dstrip) >= kDeepMinStrips;
    int cus = 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
    }
    // the two-step shape of slot k: 128-column strips where they give at least kWideMinStrips
    // strips (the launch takes them then), else 64-column strips of fstrip rows, ring of 8
    auto two_step_pick = [&](int k) {
        const int model = k < 8 ? k : LBM_STREAM_ONLY;  // slot 8: the pure pull
        const FusionPick w = wide_default(model);
        const bool wide = wide_strips(model, prec) && (long long)((nx + 2 * kStripW - 1) / (2 * kStripW)) *
                                                              ((ny + w.strip - 1) / w.strip) >= kWideMinStrips;
        return wide ? w : FusionPick{8, fstrip};
    };
    if (deep)
        for (int k = 0; k < 9; ++k) {
            const FusionPick pick = deep_pick(k < 8 ? k : LBM_STREAM_ONLY, nx, ny, prec, cus);
            ctx->fuse_depth[k] = 3;
            ctx->fuse_ring[k] = pick.ring;
            ctx->fuse_strip[k] = pick.strip;
            // a two-step launch on the three-step shape costs about what a three-step launch does
            // (measured at 4096^2 FP32, BGK: 275 us on 80-row strips against 238 us on 16-row
            // ones; at 512^2 8-row strips beat 16), so two steps left over run on 64-column strips
            // of at most the two-step default height, ring of 8 rows
            ctx->tail_ring[k] = 8;
            ctx->tail_strip[k] = fstrip > 0 ? std::min(fstrip, pick.strip) : pick.strip;
        }
    else if (fstrip > 0)
        for (int k = 0; k < 9; ++k) {
            const FusionPick t = two_step_pick(k);
            ctx->fuse_ring[k] = t.ring;
            ctx->fuse_strip[k] = t.strip;
        }
    int rc = check_hip(hipGetDevice(&ctx->device), "hipGetDevice");
    if (rc == LBM_OK) rc = scratch_address(ctx->device, &ctx->d_static);
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&ctx->d_flag, sizeof(int)), "hipMalloc(flag)");
    if (rc == LBM_OK)
        rc = check_hip(hipMalloc(&ctx->d_part, sizeof(double) * 5 * (size_t)ctx->nblocks), "hipMalloc(partials)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&ctx->d_tot, sizeof(double) * 5), "hipMalloc(totals)");
    if (rc == LBM_OK) rc = reset_flag(ctx);
    if (rc == LBM_OK) {
        LBM_DISPATCH_PREC(prec, launch_init_p, ctx, rho, ux, uy);
        rc = check_hip(hipGetLastError(), "init kernel launch");
    }
    if (rc != LBM_OK) {
        lbm_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int model, const double* omega, int nsteps) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps %d < 0", nsteps);
    int rc = validate_model(model, ctx->eq_order);
    if (rc != LBM_OK) return rc;
    rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    if (ctx->step + nsteps >= INT_MAX) return set_error(LBM_EINVAL, "step counter would overflow");
    const StepShape sh = ctx->shape_of(model);
    const int ring = ctx->fuse_ring[lbm_ctx::slot(model)], hs = ctx->fuse_strip[lbm_ctx::slot(model)];
    int s = 0;
    if ((ring == 4 || ring == 8) && ctx->fuse_depth[lbm_ctx::slot(model)] == 3)
        for (; s + 3 <= nsteps; s += 3) {
            LBM_DISPATCH_PREC(ctx->prec, launch_step3_p, ctx, model, omega, ring, hs, ctx->copy(ctx->cur),
                              ctx->copy(ctx->cur ^ 1), (int)ctx->step);
            ctx->cur ^= 1;
            ctx->step += 3;
        }
    if (ring > 0) {
        // two steps left over by three-step launches (or asked for alone): the tail shape, if any
        const bool tail = ctx->fuse_depth[lbm_ctx::slot(model)] == 3 && ctx->tail_ring[lbm_ctx::slot(model)] > 0;
        const int ring2 = tail ? ctx->tail_ring[lbm_ctx::slot(model)] : ring;
        const int hs2 = tail ? ctx->tail_strip[lbm_ctx::slot(model)] : hs;
        for (; s + 2 <= nsteps; s += 2) {
            LBM_DISPATCH_PREC(ctx->prec, launch_step2_p, ctx, model, omega, ring2, hs2, ctx->cur);
            ctx->cur ^= 1;
            ctx->step += 2;
        }
    }
    for (; s < nsteps; ++s) {
        LBM_DISPATCH_PREC(ctx->prec, launch_step_p, ctx, model, omega, sh, ctx->cur);
        ctx->cur ^= 1;
        ctx->step += 1;
    }
    return check_hip(hipGetLastError(), "step kernel launch");
}

int lbm_step_raw(lbm_ctx* ctx, int model, const double* omega, const void* src, void* dst,
                 long long step) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!src || !dst) return set_error(LBM_EINVAL, "NULL state pointer");
    if (src == dst) return set_error(LBM_EINVAL, "src and dst must differ");
    if (step < 0 || step >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step);
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    LBM_DISPATCH_PREC(ctx->prec, launch_step_raw_p, ctx, model, omega, ctx->shape_of(model), src, dst,
                      (int)step);
    return check_hip(hipGetLastError(), "raw step kernel launch");
}

int lbm_step_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src,
                      void* const* dst, int count, long long step0) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (count < 0) return set_error(LBM_EINVAL, "count %d < 0", count);
    if (count == 0) return LBM_OK;
    if (!src || !dst) return set_error(LBM_EINVAL, "NULL pointer array");
    if (step0 < 0 || step0 + count >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step0);
    for (int k = 0; k < count; ++k)
        if (!src[k] || !dst[k] || src[k] == dst[k])
            return set_error(LBM_EINVAL, "bad state pointer at step %d", k);
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    const StepShape sh = ctx->shape_of(model);
    for (int k = 0; k < count; ++k)
        LBM_DISPATCH_PREC(ctx->prec, launch_step_raw_p, ctx, model, omega, sh, src[k], dst[k], (int)(step0 + k));
    return check_hip(hipGetLastError(), "raw step kernel launch");
}

int lbm_step2_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src, void* const* mid,
                       void* const* dst, int count, long long step0) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (count < 0) return set_error(LBM_EINVAL, "count %d < 0", count);
    if (count == 0) return LBM_OK;
    if (!src || !dst) return set_error(LBM_EINVAL, "NULL pointer array");
    if (step0 < 0 || step0 + 2LL * count >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step0);
    for (int k = 0; k < count; ++k) {
        const void* m = mid ? mid[k] : nullptr;
        if (!src[k] || !dst[k] || src[k] == dst[k] || (m && (m == src[k] || m == dst[k])))
            return set_error(LBM_EINVAL, "bad state pointer at pair %d", k);
    }
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    // the raw pairs run with a ring of 8 rows: the tail strip height where the tail shape has that
    // ring, else the model's strip height
    const int slot = lbm_ctx::slot(model);
    const int fs = ctx->tail_ring[slot] == 8 ? ctx->tail_strip[slot] : ctx->fuse_strip[slot];
    const int hs = fs > 0 ? fs : 16;
    for (int k = 0; k < count; ++k)
        LBM_DISPATCH_PREC(ctx->prec, launch_step2_raw_p, ctx, model, omega, hs, src[k], mid ? mid[k] : nullptr,
                          dst[k], (int)(step0 + 2LL * k));
    return check_hip(hipGetLastError(), "raw two-step kernel launch");
}

int lbm_step3_raw_many(lbm_ctx* ctx, int model, const double* omega, const void* const* src, void* const* dst,
                       int count, long long step0) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (count < 0) return set_error(LBM_EINVAL, "count %d < 0", count);
    if (count == 0) return LBM_OK;
    if (!src || !dst) return set_error(LBM_EINVAL, "NULL pointer array");
    if (step0 < 0 || step0 + 3LL * count >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step0);
    for (int k = 0; k < count; ++k)
        if (!src[k] || !dst[k] || src[k] == dst[k]) return set_error(LBM_EINVAL, "bad state pointer at triple %d", k);
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    const int slot = lbm_ctx::slot(model);
    const int ring = ctx->fuse_ring[slot], hs = ctx->fuse_strip[slot];
    if (ctx->fuse_depth[slot] != 3 || (ring != 4 && ring != 8))
        return set_error(LBM_EUNSUPPORTED, "model %d does not take three steps per launch on this context", model);
    for (int k = 0; k < count; ++k)
        LBM_DISPATCH_PREC(ctx->prec, launch_step3_p, ctx, model, omega, ring, hs, src[k], dst[k],
                          (int)(step0 + 3LL * k));
    return check_hip(hipGetLastError(), "raw three-step kernel launch");
}

int lbm_moments(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* totals) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    LBM_DISPATCH_PREC(ctx->prec, launch_moments_p, ctx, rho, ux, uy, ctx->d_part);
    int rc = check_hip(hipGetLastError(), "moments kernel launch");
    if (rc != LBM_OK || !totals) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, ctx->stream, ctx->d_part, ctx->nblocks,
                       ctx->d_tot);
    rc = check_hip(hipGetLastError(), "finalize kernel launch");
    double t[5];
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpyAsync(t, ctx->d_tot, sizeof(t), hipMemcpyDeviceToHost, ctx->stream),
                       "copy totals");
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(ctx->stream), "synchronise");
    if (rc != LBM_OK) return rc;
    for (int k = 0; k < 4; ++k) totals[k] = t[k];
    totals[4] = t[4] / ((double)ctx->nx * (double)ctx->ny);
    totals[5] = (double)ctx->step;
    return LBM_OK;
}

int lbm_moments_noalloc(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* totals) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!ctx->d_static) return set_error(LBM_ESTATE, "context has no static scratch address");
    if (ctx->nblocks > kNoAllocMaxBlocks)
        return set_error(LBM_EINVAL, "grid %d x %d needs %d reduction blocks; lbm_moments_noalloc holds %d",
                         ctx->nx, ctx->ny, ctx->nblocks, kNoAllocMaxBlocks);
    double* part = ctx->d_static;
    double* tot = ctx->d_static + 5 * (size_t)kNoAllocMaxBlocks;
    LBM_DISPATCH_PREC(ctx->prec, launch_moments_p, ctx, rho, ux, uy, part);
    int rc = check_hip(hipGetLastError(), "moments kernel launch");
    if (rc != LBM_OK || !totals) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, ctx->stream, part, ctx->nblocks, tot);
    rc = check_hip(hipGetLastError(), "finalize kernel launch");
    if (rc != LBM_OK) return rc;
    hipLaunchKernelGGL(k_totals_out, dim3(1), dim3(64), 0, ctx->stream, tot,
                       (double)ctx->nx * (double)ctx->ny, (double)ctx->step, totals);
    return check_hip(hipGetLastError(), "totals kernel launch");
}

int lbm_status(lbm_ctx* ctx, long long* step, long long* blowup_step) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    int flag = INT_MAX;
    int rc = check_hip(hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
                       "copy blow-up flag");
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(ctx->stream), "synchronise");
    if (rc != LBM_OK) return rc;
    if (step) *step = ctx->step;
    if (blowup_step) *blowup_step = flag == INT_MAX ? -1 : (long long)flag;
    return LBM_OK;
}

int lbm_get_state(lbm_ctx* ctx, double* f) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!f) return set_error(LBM_EINVAL, "f is NULL");
    LBM_DISPATCH_PREC(ctx->prec, launch_get_p, ctx, f);
    return check_hip(hipGetLastError(), "get_state kernel launch");
}

int lbm_set_state(lbm_ctx* ctx, const double* f, long long step) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (!f) return set_error(LBM_EINVAL, "f is NULL");
    if (step < 0 || step >= INT_MAX) return set_error(LBM_EINVAL, "step %lld out of range", step);
    LBM_DISPATCH_PREC(ctx->prec, launch_set_p, ctx, f);
    int rc = check_hip(hipGetLastError(), "set_state kernel launch");
    if (rc != LBM_OK) return rc;
    ctx->step = step;
    return reset_flag(ctx);
}

int lbm_set_launch(lbm_ctx* ctx, int model, int rows, int xcd) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    int rc = validate_model(model, 4);
    if (rc != LBM_OK) return rc;
    if (rows != 1 && rows != 2 && rows != 4) return set_error(LBM_EINVAL, "rows %d not in {1,2,4}", rows);
    if (xcd != 0 && xcd != 1) return set_error(LBM_EINVAL, "xcd %d not in {0,1}", xcd);
    ctx->rows[lbm_ctx::slot(model)] = rows;
    ctx->xcd[lbm_ctx::slot(model)] = xcd;
    return LBM_OK;
}

int lbm_set_fusion(lbm_ctx* ctx, int model, int ring_rows, int strip_rows) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    int rc = validate_model(model, 4);
    if (rc != LBM_OK) return rc;
    if (ring_rows != 0 && ring_rows != 4 && ring_rows != 8 && ring_rows != 16)
        return set_error(LBM_EINVAL, "ring_rows %d not in {0, 4, 8, 16}", ring_rows);
    if (ring_rows != 0 && (strip_rows < ring_rows || strip_rows > 1 << 20 || strip_rows % ring_rows != 0))
        return set_error(LBM_EINVAL, "strip_rows %d is not a positive multiple of ring_rows %d", strip_rows,
                         ring_rows);
    ctx->fuse_ring[lbm_ctx::slot(model)] = ring_rows;
    ctx->fuse_strip[lbm_ctx::slot(model)] = ring_rows ? strip_rows : 0;
    ctx->tail_ring[lbm_ctx::slot(model)] = 0;  // an explicit shape also takes the leftover steps
    ctx->tail_strip[lbm_ctx::slot(model)] = 0;
    return LBM_OK;
}

int lbm_set_fusion_depth(lbm_ctx* ctx, int model, int steps) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    const int rc = validate_model(model, 4);  // a per-model setting, as lbm_set_fusion
    if (rc != LBM_OK) return rc;
    if (steps != 2 && steps != 3) return set_error(LBM_EINVAL, "steps per fused launch %d not in {2, 3}", steps);
    if (steps == 3 && ctx->prec == LBM_F16_SHIFTED)
        return set_error(LBM_EUNSUPPORTED, "three steps per launch need an FP32 or FP64 context");
    if (steps == 3 && (ctx->nx < 2 || ctx->ny < 2)) return set_error(LBM_EUNSUPPORTED, "grid below 2 x 2");
    ctx->fuse_depth[lbm_ctx::slot(model)] = steps;
    return LBM_OK;
}

int lbm_get_fusion_depth(lbm_ctx* ctx, int model, int* steps) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    const int rc = validate_model(model, 4);
    if (rc != LBM_OK) return rc;
    if (steps) *steps = ctx->fuse_depth[lbm_ctx::slot(model)];
    return LBM_OK;
}

int lbm_get_fusion(lbm_ctx* ctx, int model, int* ring_rows, int* strip_rows) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    int rc = validate_model(model, 4);
    if (rc != LBM_OK) return rc;
    if (ring_rows) *ring_rows = ctx->fuse_ring[lbm_ctx::slot(model)];
    if (strip_rows) *strip_rows = ctx->fuse_strip[lbm_ctx::slot(model)];
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* ctx, int model, const double* omega, int trials, int* rows_out,
                 int* xcd_out, double* us_per_step) {
    if (!ctx) return set_error(LBM_ESTATE, "context is NULL");
    if (trials < 1) return set_error(LBM_EINVAL, "trials %d < 1", trials);
    int rc = validate_model(model, ctx->eq_order);
    if (rc == LBM_OK) rc = validate_omega(omega);
    if (rc != LBM_OK) return rc;
    // the timed launches run ahead of the step counter and may record a blow-up of a step not
    // taken yet: the record is restored afterwards
    int flag0 = 0;
    rc = check_hip(hipMemcpyAsync(&flag0, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
                   "hipMemcpyAsync(flag)");
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (rc != LBM_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (rc == LBM_OK) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
    // times `trials` launches of `launch` after one untimed one; milliseconds
    auto timed = [&](auto&& launch) -> float {
        launch();
        if (rc == LBM_OK) rc = check_hip(hipEventRecord(e0, ctx->stream), "hipEventRecord");
        for (int t = 0; t < trials && rc == LBM_OK; ++t) launch();
        if (rc == LBM_OK) rc = check_hip(hipGetLastError(), "autotune launch");
        if (rc == LBM_OK) rc = check_hip(hipEventRecord(e1, ctx->stream), "hipEventRecord");
        if (rc == LBM_OK) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        if (rc == LBM_OK) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms;
    };
    // every launch recomputes from copy `cur` into the other copy: state and counter unchanged
    const int rows_c[3] = {1, 2, 4};
    float best = 0.f;
    int best_rows = ctx->rows[lbm_ctx::slot(model)], best_xcd = ctx->xcd[lbm_ctx::slot(model)];
    for (int ri = 0; ri < 3 && rc == LBM_OK; ++ri)
        for (int xi = 0; xi < 2 && rc == LBM_OK; ++xi) {
            const StepShape sh = step_shape(ctx->nx, ctx->ny, rows_c[ri], xi);
            const float ms = timed([&] { LBM_DISPATCH_PREC(ctx->prec, launch_step_p, ctx, model, omega, sh, ctx->cur); });
            if (rc == LBM_OK && (best == 0.f || ms < best)) {
                best = ms;
                best_rows = rows_c[ri];
                best_xcd = xi;
            }
        }
    const float best1 = best;  // the best single-step shape, per step
    // two-step shapes, per step
    const int fuse_c[8][2] = {{8, 8}, {8, 16}, {8, 40}, {8, 64}, {16, 16}, {4, 16}, {4, 20}, {4, 64}};
    int best_ring = 0, best_strip = 0, best_depth = 2;
    float best2 = 0.f;  // the fastest two-step shape: the tail shape of three-step runs
    int tail_ring = 0, tail_strip = 0;
    for (int k = 0; k < 8 && rc == LBM_OK; ++k) {
        const int ring = fuse_c[k][0], hs = fuse_c[k][1];
        const float ms = 0.5f * timed([&] { LBM_DISPATCH_PREC(ctx->prec, launch_step2_p, ctx, model, omega, ring, hs, ctx->cur); });
        if (rc == LBM_OK && ms < best) {
            best = ms;
            best_ring = ring;
            best_strip = hs;
        }
        if (rc == LBM_OK && (best2 == 0.f || ms < best2)) {
            best2 = ms;
            tail_ring = ring;
            tail_strip = hs;
        }
    }
    // three-step shapes, per step (not for FP16 or grids below 2 x 2)
    const int deep_c[12][2] = {{4, 8}, {4, 16}, {4, 32}, {4, 64}, {8, 8}, {8, 16}, {8, 24}, {8, 32},
                               {8, 64}, {8, 80}, {8, 96}, {8, 128}};
    for (int k = 0; k < 12 && rc == LBM_OK && ctx->prec != LBM_F16_SHIFTED && ctx->nx >= 2 && ctx->ny >= 2; ++k) {
        const int ring = deep_c[k][0], hs = deep_c[k][1];
        const float ms = timed([&] {
            LBM_DISPATCH_PREC(ctx->prec, launch_step3_p, ctx, model, omega, ring, hs, ctx->copy(ctx->cur),
                              ctx->copy(ctx->cur ^ 1), (int)ctx->step);
        }) / 3.f;
        if (rc == LBM_OK && ms < best) {
            best = ms;
            best_ring = ring;
            best_strip = hs;
            best_depth = 3;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpyAsync(ctx->d_flag, &flag0, sizeof(int), hipMemcpyHostToDevice, ctx->stream),
                       "hipMemcpyAsync(flag)");
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (rc != LBM_OK) return rc;
    ctx->rows[lbm_ctx::slot(model)] = best_rows;
    ctx->xcd[lbm_ctx::slot(model)] = best_xcd;
    ctx->fuse_ring[lbm_ctx::slot(model)] = best_ring;
    ctx->fuse_strip[lbm_ctx::slot(model)] = best_strip;
    ctx->fuse_depth[lbm_ctx::slot(model)] = best_depth;
    // the fastest two-step shape takes the two steps left after three-step launches, if it beats
    // one step per launch
    const bool tail = best_depth == 3 && best_ring > 0 && tail_ring > 0 && best2 < best1;
    ctx->tail_ring[lbm_ctx::slot(model)] = tail ? tail_ring : 0;
    ctx->tail_strip[lbm_ctx::slot(model)] = tail ? tail_strip : 0;
    if (rows_out) *rows_out = best_rows;
    if (xcd_out) *xcd_out = best_xcd;
    if (us_per_step) *us_per_step = 1e3 * (double)best / trials;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->d_flag) (void)hipFree(ctx->d_flag);
    if (ctx->d_part) (void)hipFree(ctx->d_part);
    if (ctx->d_tot) (void)hipFree(ctx->d_tot);
    if (ctx->d_wslots) (void)hipFree(ctx->d_wslots);
    delete ctx;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
