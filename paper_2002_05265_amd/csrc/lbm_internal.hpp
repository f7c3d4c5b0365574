// Internal helpers of liblbm shared by the plain, batched and adjoint kernels: storage types,
// periodic neighbour addressing, pull loads / stores, conserved quantities, block reductions
// and the context structure behind the opaque lbm_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "lbm.h"
#include "lbm_cell.hpp"

#ifndef LBM_DEFAULT_ROWS
#define LBM_DEFAULT_ROWS 1
#endif
#ifndef LBM_DEFAULT_XCD
#define LBM_DEFAULT_XCD 0
#endif

namespace lbm {

// Storage type S and arithmetic type R of each precision.
template <int PREC> struct Store;
template <> struct Store<kF64> { using S = double; using R = double; };
template <> struct Store<kF32> { using S = float; using R = float; };
template <> struct Store<kF16> { using S = _Float16; using R = float; };

inline size_t elem_size(int prec) { return prec == LBM_F64 ? 8 : (prec == LBM_F32_SHIFTED ? 4 : 2); }

struct Geom {
    int nx, ny;
    long long plane;  // elements per population plane
};

struct Launch {
    dim3 grid, block;
};

// Launch shape of the step kernels: bw x bh threads, each thread `rows` nodes along y, gx x gy
// tiles launched as a 1D grid (optionally renumbered per XCD).
struct StepShape {
    int bw, bh, rows, xcd;
    unsigned gx, gy;
};

// Row offsets of rows y, y-1, y+1 and columns x, x-1, x+1 with periodic wrap.
struct Nbr {
    unsigned r0, rm, rp;
    unsigned x, xm, xp;
};

__device__ __forceinline__ Nbr neighbours(int x, int y, int nx, int ny) {
    Nbr n;
    // one per-lane multiply; the wrapped rows come from the wave-uniform (ny - 1) nx
    n.r0 = (unsigned)y * (unsigned)nx;
    n.rm = y == 0 ? (unsigned)(ny - 1) * (unsigned)nx : n.r0 - (unsigned)nx;
    n.rp = y == ny - 1 ? 0u : n.r0 + (unsigned)nx;
    n.x = (unsigned)x;
    n.xm = (unsigned)(x == 0 ? nx - 1 : x - 1);
    n.xp = (unsigned)(x == nx - 1 ? 0 : x + 1);
    return n;
}

// Streaming loads / stores of population data.  Every population is read once and written
// once per step, so the non-temporal variants keep it from displacing reusable lines.
#ifndef LBM_NT_LOADS
#define LBM_NT_LOADS 0
#endif
#ifndef LBM_NT_STORES
#define LBM_NT_STORES 1
#endif

template <typename S>
__device__ __forceinline__ S ld(const S* p) {
#if LBM_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <typename S, bool NT = (LBM_NT_STORES != 0)>
__device__ __forceinline__ void st(S* p, S v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Address of the element at byte offset `off` (< 2^31) of plane q.  The plane base is the same
// for the whole wave (scalar registers) and the per-lane part stays a 32-bit byte offset, so the
// access needs no 64-bit address arithmetic per lane (global loads and stores take a scalar base
// plus a 32-bit vector offset).
template <typename S>
__device__ __forceinline__ S* plane_at(S* base, long long plane, int q, unsigned off) {
    using B = typename std::conditional<std::is_const<S>::value, const char, char>::type;
    return reinterpret_cast<S*>(reinterpret_cast<B*>(base + q * plane) + off);
}

// Gather f_i(x) = stored_i(x - xi_i).
template <typename S, typename R>
__device__ __forceinline__ void pull_load(const S* __restrict__ src, long long plane, const Nbr& n,
                                          R (&h)[9]) {
    constexpr unsigned E = sizeof(S);
    const unsigned r0 = n.r0 * E, rm = n.rm * E, rp = n.rp * E;
    const unsigned x0 = n.x * E, xm = n.xm * E, xp = n.xp * E;
    h[0] = R(ld(plane_at(src, plane, 0, r0 + x0)));
    h[1] = R(ld(plane_at(src, plane, 1, r0 + xm)));
    h[2] = R(ld(plane_at(src, plane, 2, rm + x0)));
    h[3] = R(ld(plane_at(src, plane, 3, r0 + xp)));
    h[4] = R(ld(plane_at(src, plane, 4, rp + x0)));
    h[5] = R(ld(plane_at(src, plane, 5, rm + xm)));
    h[6] = R(ld(plane_at(src, plane, 6, rm + xp)));
    h[7] = R(ld(plane_at(src, plane, 7, rp + xp)));
    h[8] = R(ld(plane_at(src, plane, 8, rp + xm)));
}

// Conversion to the storage type.  For FP16 the value is first materialised as an FP32
// register (an empty asm with a register constraint): otherwise the compiler may fuse the last
// FMA with the rounding to half in one kernel and not in another, and the batched, plain and
// adjoint kernels would round differently.
template <typename S, typename R>
__device__ __forceinline__ S to_store(R v) {
    if constexpr (std::is_same<S, _Float16>::value) {
        float f = (float)v;
        asm volatile("" : "+v"(f));
        return (S)f;
    } else {
        return (S)v;
    }
}

template <typename S, typename R, bool NT = (LBM_NT_STORES != 0)>
__device__ __forceinline__ void store_cell(S* __restrict__ dst, long long plane, unsigned c,
                                           const R (&h)[9]) {
    const unsigned off = c * (unsigned)sizeof(S);
#pragma unroll
    for (int i = 0; i < 9; ++i) st<S, NT>(plane_at(dst, plane, i, off), to_store<S>(h[i]));
}

// Tile of a 1D-launched block.  The hardware hands consecutive block ids to the eight XCDs in
// turn; with `xcd` set, the ids are renumbered so that each XCD owns one contiguous band of
// tiles (neighbouring tiles then share their edge cache lines in the same L2).
__device__ __forceinline__ void tile_of_block(unsigned b, unsigned gx, unsigned nb, int xcd,
                                              unsigned& bx, unsigned& by) {
    if (xcd) {
        const unsigned per = nb >> 3, rem = nb & 7u, k = b & 7u, j = b >> 3;
        b = k * per + (k < rem ? k : rem) + j;
    }
    by = b / gx;
    bx = b - by * gx;
}

// Strip (bx, by) of block b of a launch over nb = sx * sy strips, the strips taken in groups of G
// adjacent strip columns (group-major, row-major inside a group) and that order dealt to the XCDs
// in contiguous bands (the hardware hands block b to XCD b mod 8): each XCD walks whole column
// groups from top to bottom, so neighbouring strips run at the same time on one XCD and share the
// lines at their common edge in its L2, while the XCDs together sweep the same rows of the grid.
__device__ __forceinline__ void strip_of_block_grouped(unsigned b, unsigned sx, unsigned nb, unsigned G,
                                                       unsigned& bx, unsigned& by) {
    const unsigned per = nb >> 3, rem = nb & 7u, k = b & 7u, j = b >> 3;
    const unsigned t = k * per + (k < rem ? k : rem) + j;  // position in group-major order
    const unsigned sy = nb / sx;
    const unsigned g = t / (G * sy), r = t - g * (G * sy);
    const unsigned gw = min(G, sx - g * G);
    by = r / gw;
    bx = g * G + (r - by * gw);
}

// Store value i of node (x, y) where the next pull of node (x, y) reads it, i.e. at node
// (x, y) - xi_i: the buffer then holds the state pre-streamed backwards by one step.
template <typename S, typename R>
__device__ __forceinline__ void prestream_store(S* __restrict__ dst, const Geom& g, int x, int y,
                                                const R (&h)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xd = x - cx(i), yd = y - cy(i);
        xd = xd < 0 ? g.nx - 1 : (xd >= g.nx ? 0 : xd);
        yd = yd < 0 ? g.ny - 1 : (yd >= g.ny ? 0 : yd);
        dst[i * g.plane + (long long)yd * g.nx + xd] = to_store<S>(h[i]);
    }
}

// Conserved quantities of a cell: rho = rho_s + sum_i h_i, u = U + (j_h - delta rho U) / rho.
// For FP32 storage the nine-term mass sum is carried in FP64 (delta rho ~ 1e-4 of rho needs more
// than FP32's 24 bits once added to rho_s); for binary16 storage the rounding of the stored values
// (2^-11 |h|) is far above that of an FP32 sum, which is used there.  rho_d returns rho for the
// blow-up test.  S is the storage type.
template <typename S, typename R>
__device__ __forceinline__ Macro<R> macro_of(const R (&h)[9], const Ref<R>& ref, double& rho_d) {
    Macro<R> m;
    if constexpr (std::is_same<R, double>::value || std::is_same<S, _Float16>::value) {
        m.drho = ((h[0] + (h[1] + h[3])) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8]));
        m.rho = ref.rho + m.drho;
        rho_d = m.rho;
    } else {
        const double d = (((double)h[0] + ((double)h[1] + (double)h[3])) + ((double)h[2] + (double)h[4])) +
                         (((double)h[5] + (double)h[7]) + ((double)h[6] + (double)h[8]));
        rho_d = (double)ref.rho + d;
        m.drho = (R)d;
        m.rho = (R)rho_d;
    }
    m.jx = ((h[1] + h[5]) + h[8]) - ((h[3] + h[6]) + h[7]);
    m.jy = ((h[2] + h[5]) + h[6]) - ((h[4] + h[7]) + h[8]);
    // FP32 arithmetic takes the hardware reciprocal (1 ulp; the correctly rounded quotient costs
    // nine more instructions per node): it scales O(u) quantities only, and every kernel that
    // collides (plain, batched, adjoint) shares this function, so they stay bit-identical
    if constexpr (std::is_same<R, float>::value)
        m.inv_rho = __builtin_amdgcn_rcpf(m.rho);
    else
        m.inv_rho = R(1) / m.rho;
    m.dux = (m.jx - m.drho * ref.ux) * m.inv_rho;
    m.duy = (m.jy - m.drho * ref.uy) * m.inv_rho;
    m.ux = ref.ux + m.dux;
    m.uy = ref.uy + m.duy;
    return m;
}

// Conserved quantities of a node given by its macroscopic fields (FP64, initialisation).
__host__ __device__ inline Macro<double> macro_of_fields(double rho, double ux, double uy,
                                                         const Ref<double>& r) {
    Macro<double> m;
    m.rho = rho;
    m.ux = ux;
    m.uy = uy;
    m.drho = rho - r.rho;
    m.dux = ux - r.ux;
    m.duy = uy - r.uy;
    m.jx = rho * ux - r.rho * r.ux;
    m.jy = rho * uy - r.rho * r.uy;
    m.inv_rho = 1.0 / rho;
    return m;
}

// Stored deviations of f^eq_N(rho, u) with respect to the reference (FP64).
__host__ __device__ inline void eq_deviation(double rho, double ux, double uy, const Ref<double>& r,
                                             int N, double (&h)[9]) {
    const Macro<double> m = macro_of_fields(rho, ux, uy, r);
    const Eq<double> e = hermite_eq(m, r, N);
    hermite_to_pop(m, e.e20, e.e02, e.e11, e.e21, e.e12, e.e22, h);
}

// The nine reference populations f^eq_N(rho_s, U) (FP64), added back by get_state.
struct Pop9 {
    double v[9];
};

inline Pop9 reference_populations(const Ref<double>& r, int N) {
    const Ref<double> zero{0.0, 0.0, 0.0};
    double h[9];
    eq_deviation(r.rho, r.ux, r.uy, zero, N, h);
    Pop9 p;
    for (int i = 0; i < 9; ++i) p.v[i] = h[i];
    return p;
}

// Reference of a precision: none for FP64; for shifted storage the values are rounded to FP32
// once so that the FP32 kernels and the FP64 set-up use exactly the same reference.
inline Ref<double> storage_reference(int prec, double rho0, double ux0, double uy0) {
    if (prec == LBM_F64) return Ref<double>{0.0, 0.0, 0.0};
    return Ref<double>{(double)(float)rho0, (double)(float)ux0, (double)(float)uy0};
}

template <typename R>
inline Ref<R> ref_as(const Ref<double>& r) {
    return Ref<R>{(R)r.rho, (R)r.ux, (R)r.uy};
}

// Record `step` in *flag (atomic min) if any lane of the wave saw a bad node.
__device__ __forceinline__ void flag_bad(bool bad, int* flag, int step) {
    const unsigned long long b = __ballot(bad);
    if (b != 0ull) {
        const int first = __ffsll((unsigned long long)b) - 1;
        if ((int)__lane_id() == first) atomicMin(flag, step);
    }
}

// Sum K doubles over the block (any 1D/2D shape up to 1024 threads) and write them to out[]
// from thread 0.  Fixed reduction order: deterministic.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* __restrict__ out) {
    __shared__ double sh[16][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0)
        for (int k = 0; k < K; ++k) sh[wave][k] = v[k];
    __syncthreads();
    if (tid == 0) {
        const int nw = (nthreads + 63) >> 6;
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[w][k];
            out[k] = s;
        }
    }
}

int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
Launch launch_for(int nx, int ny);
StepShape step_shape(int nx, int ny, int rows, int xcd);
long long plane_elems(int nx, int ny, int prec);
int validate_omega(const double* w);
int validate_model(int model, int eq_order);

}  // namespace lbm

struct lbm_ctx;
namespace lbm {
int reset_blowup(lbm_ctx* ctx);     // blow-up record := none (kernel on the context's stream)
int reduce_partials(lbm_ctx* ctx);  // d_tot[0..4] := sum over blocks of d_part (fixed order)
}  // namespace lbm

struct lbm_ctx {
    int nx = 0, ny = 0, prec = 0, eq_order = 4;
    lbm::Ref<double> ref{0.0, 0.0, 0.0};  // storage reference: h_i = f_i - f^eq_N(rho_s, U)_i
    lbm::Pop9 fref{};                      // the reference populations
    char* buf = nullptr;          // caller-owned population buffer (two copies)
    size_t bytes = 0;
    long long plane = 0;          // elements per population plane
    size_t esize = 8;             // bytes per stored population
    int cur = 0;                  // copy holding f*(., n - 1)
    long long step = 0;           // n
    hipStream_t stream = nullptr;
    int device = 0;
    int nblocks = 0;              // blocks of the per-cell launch
    int* d_flag = nullptr;        // first bad step (INT_MAX = none)
    double* d_part = nullptr;     // per-block partial sums, 5 per block (reduction scratch)
    double* d_tot = nullptr;      // 5 totals
    double* d_static = nullptr;   // this device's address of the library's static reduction scratch
    double* d_wslots = nullptr;   // adjoint: per-block pending rate-gradient sums, 5 per block
    bool wslots_live = false;     // d_wslots holds pending sums
    int adj_depth = 1;            // reverse steps per launch in lbm_adjoint_many (1 or 2)

    int rows[9] = {LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS,
                   LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS, LBM_DEFAULT_ROWS,
                   LBM_DEFAULT_ROWS};   // nodes per thread along y, per model (index 8: stream)
    int xcd[9] = {LBM_DEFAULT_XCD, LBM_DEFAULT_XCD, LBM_DEFAULT_XCD, LBM_DEFAULT_XCD,
                  LBM_DEFAULT_XCD, LBM_DEFAULT_XCD, LBM_DEFAULT_XCD, LBM_DEFAULT_XCD,
                  LBM_DEFAULT_XCD};     // XCD-banded tile order, per model

    int fuse_ring[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // two steps per pass: ring rows (0 = off)
    int fuse_strip[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // and strip height, per model
    int fuse_depth[9] = {2, 2, 2, 2, 2, 2, 2, 2, 2};  // steps per fused launch (2 or 3)
    // the two-step launch that ends a run of three-step launches (two steps left): its own ring
    // and strip height (0: those of fuse_ring / fuse_strip)
    int tail_ring[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int tail_strip[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

    static int slot(int model) { return (model >= 0 && model < 8) ? model : 8; }
    lbm::StepShape shape_of(int model) const {
        return lbm::step_shape(nx, ny, rows[slot(model)], xcd[slot(model)]);
    }
    char* copy(int c) const { return buf + (size_t)c * 9 * (size_t)plane * esize; }
    lbm::Geom geom() const { return lbm::Geom{nx, ny, plane}; }
};
