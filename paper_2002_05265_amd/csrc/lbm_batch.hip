// Batched stability sweep: many independent D2Q9 runs advanced by one persistent launch.
//
// Work decomposition.  Instance j owns `cells_j = nx_j * ny_j` nodes, cut into tiles of
// 256 * NPT consecutive nodes (linear index y * nx + x).  All tiles of all instances form one
// list per XCD (every instance is owned by one XCD); a persistent grid of workgroups, launched
// cooperatively and sized to what really stays co-resident, takes on each XCD the tiles of that
// XCD's list, then the workgroups of the XCD meet at a barrier before the next step reads what
// this one wrote (see the XCD-local execution notes below).  Barriers are monotonic counters,
// and every spin is bounded in wall-clock time, so every wave exits whatever happens to others.
//
// Each node runs exactly the code of the plain kernel (pull_load / macro_of / collide /
// store_cell with the same coefficients), so an instance is bit-identical to its plain run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_batch.h"
#include "lbm_cell.hpp"
#include "lbm_internal.hpp"
#include "lbm_step2.hpp"
#include "lbm_step3.hpp"

using namespace lbm;

namespace {

constexpr int kTileThreads = 256;

template <typename R>
struct BDesc {
    int nx, ny, model, N;
    int cells, tile0;       // node count, first tile of this instance (for the current NPT)
    long long off;          // element offset of the instance inside each copy
    long long plane;        // elements per population plane of the instance
    long long foff;         // offset of the instance's initial fields
    float inv_nx;
    Ref<R> ref;             // storage reference (rho_s, U) in the arithmetic type
    Ref<double> ref_d;      // the same values in FP64 (initialisation)
    Coef<R> c;
};

__device__ __forceinline__ int row_of(int c, int nx, float inv_nx) {
    int y = (int)((float)c * inv_nx);
    if (y * nx > c) --y;
    else if ((y + 1) * nx <= c) ++y;
    return y;
}

template <typename R>
__device__ __forceinline__ void collide_model(int model, R (&h)[9], const Macro<R>& m,
                                              const Ref<R>& r, const Coef<R>& c, int N) {
    switch (model) {
        case kBGK: collide<kBGK>(h, m, r, c, N); break;
        case kRM: collide<kRM>(h, m, r, c, N); break;
        case kHM: collide<kHM>(h, m, r, c, N); break;
        case kCM: collide<kCM>(h, m, r, c, N); break;
        case kCHM: collide<kCHM>(h, m, r, c, N); break;
        case kK: collide<kK>(h, m, r, c, N); break;
        case kPR: collide<kPR>(h, m, r, c, N); break;
        default: collide<kRR>(h, m, r, c, N); break;
    }
}

// XCD-local execution.  MI355X has one L2 per XCD and the eight L2s are not coherent with each
// other, so a grid-wide barrier needs agent-scope fences that write back and invalidate a whole L2
// per workgroup and step (measured: ~55 us per step for the fences alone).  Instead, every
// instance is owned by one XCD: the host deals instances to the XCDs and builds one tile list per
// XCD, each workgroup reads the XCD it runs on from the hardware (XCC_ID) and only works on that
// XCD's tiles, and the workgroups of one XCD meet at their own barrier each step.  All data a
// workgroup reads were then written through the same L2, so release is "my stores have reached
// the L2" (s_waitcnt vmcnt(0)) and the acquire side is that the population loads of this kernel
// are agent-scope loads, which never hit in the CU's L1 (a workgroup-scope L1 invalidate,
// buffer_inv sc0, was measured to leave stale lines outside thread-group-split mode, and an
// agent-scope invalidate costs ~30 us per step).  The stores of this kernel are plain (no
// non-temporal hint), so every line goes through the shared L2.
//
// Barrier words, 256-byte lines of 64 unsigned: line 0 counts all workgroups at launch, line
// 1 + x counts the workgroups on XCD x, line 1 + kMaxXcc + x is XCD x's step barrier.
constexpr int kMaxXcc = 16;
constexpr int kLine = 64;
constexpr int kBarrierWords = kLine * (1 + 2 * kMaxXcc);

__device__ __forceinline__ unsigned xcc_id() {
    // hwreg(HW_REG_XCC_ID, 0, 4): bits 3:0 of hardware register 20
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kMaxXcc - 1);
}

// SGPRs per wave that each persistent kernel is compiled to at most (amdgpu_num_sgpr), and the
// waves per SIMD that leaves.  Measured on MI355X: kernels of 24, 82, 92 and 106 SGPRs held 8, 7, 7
// and 6 waves per SIMD, one fewer than the usual rule of 800 SGPRs in granules of 16 that the
// compiler's and the runtime's occupancy figures apply (both report 8, 8, 8, 7): a wave occupies
// roundup(S, 16) + 16 of the SIMD's 800.  The one-step FP32 / FP16 kernel is held to 80 SGPRs (it
// would take 82, and so 7 waves per SIMD); the others are limited by VGPRs or LDS well below their
// SGPR figure.
template <int PREC> constexpr int batch1_sgprs() { return PREC == kF64 ? 112 : 80; }  // k_batch64 / k_batch
constexpr int kBatchFusedSgprs = 112;                                                  // k_batch2, k_batch3
constexpr int sgpr_waves(int sgprs) {
    return std::min(8, 800 / ((sgprs + 15) / 16 * 16 + 16));
}

// Spin (thread 0 of a workgroup) until *ctr >= target, or until err is set or the wall-clock
// bound passes (then err = 1).  Returns false if the launch must stop.
__device__ __forceinline__ bool wait_count(const unsigned* ctr, unsigned target, int* err, long long timeout_ticks) {
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (wall_clock64() - t0 > timeout_ticks) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Barrier of the `count` workgroups of one XCD after step s (counter target (s + 1) count).
__device__ __forceinline__ bool xcd_barrier(unsigned* ctr, int step, unsigned count, int* err,
                                            long long timeout_ticks) {
    __shared__ int ok;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = wait_count(ctr, ((unsigned)step + 1u) * count, err, timeout_ticks) ? 1 : 0;
    }
    __syncthreads();
    return ok != 0;
}

// Registration of a workgroup of the persistent grid: its rank among the workgroups on its XCD
// and their count, once every workgroup of the grid has registered, and the step counter at the
// launch start.  The counter is read before this workgroup registers: block 0 advances it when it
// has finished all its passes, and since its barriers wait only for its own XCD, a workgroup that
// read the counter after registering could read the advanced value (and take the wrong copy and
// steps).  False if the launch must stop (a bound passed, or an XCD that owns work got no
// workgroup: err = 2).
__device__ __forceinline__ bool register_group(unsigned* __restrict__ bar, const int* __restrict__ xtab,
                                               int* __restrict__ err, long long timeout_ticks, unsigned xcc,
                                               const long long* __restrict__ step_ctr, unsigned& rank,
                                               unsigned& count, long long& n0) {
    __shared__ unsigned s_rank, s_count;
    __shared__ int s_go;
    __shared__ long long s_n0;
    if (threadIdx.x == 0) {
        s_n0 = __hip_atomic_load(step_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // (the s_waitcnt below completes this load before the grid count is incremented)
        s_rank = __hip_atomic_fetch_add(bar + kLine * (1 + xcc), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the XCD count must be complete before the grid count is: wait until this add has been
        // performed (it returns) before issuing the next one, so that whoever sees the grid count
        // at gridDim.x reads final XCD counts
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int go = wait_count(bar, gridDim.x, err, timeout_ticks) ? 1 : 0;
        s_count = __hip_atomic_load(bar + kLine * (1 + xcc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // an XCD that owns tiles but got no workgroup would leave its instances behind
        for (int x = 0; x < kMaxXcc && go; ++x)
            if (xtab[2 * x + 1] > 0 &&
                __hip_atomic_load(bar + kLine * (1 + x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                go = 0;
            }
        s_go = go;
    }
    __syncthreads();
    rank = s_rank;
    count = s_count;
    n0 = s_n0;
    return s_go != 0;
}

template <int PREC, int NPT>
__device__ __forceinline__ void batch_steps(
    typename Store<PREC>::S* __restrict__ base, long long copy_elems,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int2* __restrict__ run,
    const int* __restrict__ xtab, int* __restrict__ blowup, const int* __restrict__ active,
    int* __restrict__ lastcopy, unsigned* __restrict__ bar, int* __restrict__ err,
    long long* __restrict__ step_ctr, int nsteps, int advance, long long timeout_ticks) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    const int tid = threadIdx.x;
    const unsigned xcc = xcc_id();
    unsigned rank, count;
    long long n0;
    if (!register_group(bar, xtab, err, timeout_ticks, xcc, step_ctr, rank, count, n0)) return;
    const int first_tile = xtab[2 * xcc], ntiles = xtab[2 * xcc + 1];
    unsigned* xbar = bar + kLine * (1 + kMaxXcc + xcc);
    for (int s = 0; s < nsteps; ++s) {
        const long long n = n0 + (advance ? s : 0);
        const int sc = (int)(n & 1);
        const S* src = base + sc * copy_elems;
        S* dst = base + (sc ^ 1) * copy_elems;
        for (int t = (int)rank; t < ntiles; t += (int)count) {
            const int2 e = run[first_tile + t];  // (instance, tile within the instance)
            const int j = e.x;
            const BDesc<R>& d = desc[j];
            const int frozen = __hip_atomic_load(blowup + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((long long)frozen < n || !active[j]) continue;  // blew up earlier, or retired
            if (advance && e.y == 0 && tid == 0) lastcopy[j] = sc ^ 1;
            const int first = e.y * NPT * kTileThreads + tid;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int c = first + k * kTileThreads;
                if (c < d.cells) {
                    const int y = row_of(c, d.nx, d.inv_nx);
                    const int x = c - y * d.nx;
                    const Nbr nb = neighbours(x, y, d.nx, d.ny);
                    R h[9];
                    pull_load_l2(src + d.off, d.plane, nb, h);
                    double rho_d;
                    const Macro<R> m = macro_of<S>(h, d.ref, rho_d);
                    flag_bad(!(rho_d > 0.0), blowup + j, (int)n);
                    collide_model(d.model, h, m, d.ref, d.c, d.N);
                    store_cell<S, R, false>(dst + d.off, d.plane, (unsigned)c, h);
                }
            }
        }
        if (!xcd_barrier(xbar, s, count, err, timeout_ticks)) return;
    }
    if (advance && blockIdx.x == 0 && tid == 0) *step_ctr = n0 + nsteps;
}

// The one-step persistent kernel: FP32 / FP16 held to 80 SGPRs (8 waves per SIMD), FP64 to 112.
template <int PREC, int NPT>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_num_sgpr(80))) void k_batch(
    typename Store<PREC>::S* __restrict__ base, long long copy_elems,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int2* __restrict__ run,
    const int* __restrict__ xtab, int* __restrict__ blowup, const int* __restrict__ active,
    int* __restrict__ lastcopy, unsigned* __restrict__ bar, int* __restrict__ err,
    long long* __restrict__ step_ctr, int nsteps, int advance, long long timeout_ticks) {
    batch_steps<PREC, NPT>(base, copy_elems, desc, run, xtab, blowup, active, lastcopy, bar, err, step_ctr, nsteps, advance, timeout_ticks);
}

template <int NPT, int PREC = kF64>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_num_sgpr(112))) void k_batch64(
    typename Store<PREC>::S* __restrict__ base, long long copy_elems,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int2* __restrict__ run,
    const int* __restrict__ xtab, int* __restrict__ blowup, const int* __restrict__ active,
    int* __restrict__ lastcopy, unsigned* __restrict__ bar, int* __restrict__ err,
    long long* __restrict__ step_ctr, int nsteps, int advance, long long timeout_ticks) {
    batch_steps<PREC, NPT>(base, copy_elems, desc, run, xtab, blowup, active, lastcopy, bar, err, step_ctr, nsteps, advance, timeout_ticks);
}

// The one-step kernel of a precision.
template <int PREC, int NPT>
const void* batch1_fn() {
    if constexpr (PREC == kF64)
        return reinterpret_cast<const void*>(&k_batch64<NPT>);
    else
        return reinterpret_cast<const void*>(&k_batch<PREC, NPT>);
}

// Two steps per pass: the same persistent grid and XCD-local barriers as k_batch, one barrier
// per pair of steps, over strips of kStripW columns and `hs` rows of the instances (the strip
// body of the plain two-step kernel, with loads that bypass L1 and plain stores).  Pair p of a
// launch reads the copy of its first step's parity at the launch start, flipped p times, so
// after an even number of pairs every live instance's state is back in the copy of its step's
// parity.  Whether a strip is skipped (its instance blew up before the pair, or was retired)
// is decided once per workgroup: the strip body contains block barriers.
template <int PREC, int RING>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_num_sgpr(112))) void k_batch2(
    typename Store<PREC>::S* __restrict__ base, long long copy_elems,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int2* __restrict__ run,
    const int* __restrict__ xtab, int* __restrict__ blowup, const int* __restrict__ active,
    int* __restrict__ lastcopy, unsigned* __restrict__ bar, int* __restrict__ err,
    long long* __restrict__ step_ctr, int npairs, int advance, long long timeout_ticks, int hs) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    __shared__ S ring[9][RING + 2][kStripW + 2];
    __shared__ int s_skip;
    const int tid = threadIdx.x;
    const unsigned xcc = xcc_id();
    unsigned rank, count;
    long long n0;
    if (!register_group(bar, xtab, err, timeout_ticks, xcc, step_ctr, rank, count, n0)) return;
    const int first_strip = xtab[2 * xcc], nstrips = xtab[2 * xcc + 1];
    unsigned* xbar = bar + kLine * (1 + kMaxXcc + xcc);
    for (int p = 0; p < npairs; ++p) {
        const long long n = n0 + (advance ? 2 * p : 0);
        const int sc = (int)(n0 & 1) ^ (advance ? (p & 1) : 0);
        const S* src = base + sc * copy_elems;
        S* dst = base + (sc ^ 1) * copy_elems;
        for (int t = (int)rank; t < nstrips; t += (int)count) {
            const int2 e = run[first_strip + t];  // (instance, strip within the instance)
            const int j = e.x;
            const BDesc<R>& d = desc[j];
            if (tid == 0) {
                const int frozen = __hip_atomic_load(blowup + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_skip = ((long long)frozen < n || !active[j]) ? 1 : 0;  // blew up earlier, or retired
                if (!s_skip && advance && e.y == 0) lastcopy[j] = sc ^ 1;
            }
            __syncthreads();
            const bool skip = s_skip != 0;
            __syncthreads();  // s_skip is rewritten for the next strip only after every thread read it
            if (skip) continue;
            const int gsx = (d.nx + kStripW - 1) / kStripW;
            const int sy = e.y / gsx;
            const int x0 = (e.y - sy * gsx) * kStripW, ys = sy * hs;
            const Geom g{d.nx, d.ny, d.plane};
            strip_two_steps<RING, kStripW, true, false>(ring, src + d.off, dst + d.off, g, d.ref, x0, ys, min(ys + hs, d.ny),
                                               (int)n, blowup + j, [&](R(&h)[9], const Macro<R>& m) {
                                                   collide_model(d.model, h, m, d.ref, d.c, d.N);
                                               });
        }
        if (!xcd_barrier(xbar, p, count, err, timeout_ticks)) return;
    }
    if (advance && blockIdx.x == 0 && tid == 0) *step_ctr = n0 + 2LL * npairs;
}

// Strip width of the FP64 three-step batched kernel: the strip and its halo fit one wave.
constexpr int kBatchNarrowW = 48;

// Three steps per pass: the same persistent grid and XCD-local barriers as k_batch2, with the strip
// body of the plain three-step kernels (two LDS rings of RING + 2 rows): in FP64 the narrow strips
// of 48 columns whose halo fits the wave, in FP32 strips of 64 columns (its own strip table).  A
// triple changes both the step's parity and the copy, so triple p of a launch reads the copy of its
// first step's parity (the copy of the launch start, flipped p times) and any number of triples
// keeps every live state in the copy of its step's parity.
template <int PREC, int RING>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_num_sgpr(112))) void k_batch3(
    typename Store<PREC>::S* __restrict__ base, long long copy_elems,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int2* __restrict__ run,
    const int* __restrict__ xtab, int* __restrict__ blowup, const int* __restrict__ active,
    int* __restrict__ lastcopy, unsigned* __restrict__ bar, int* __restrict__ err,
    long long* __restrict__ step_ctr, int ntriples, int advance, long long timeout_ticks, int hs) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    constexpr bool NARROW = PREC == kF64;
    constexpr int SW = NARROW ? kBatchNarrowW : kStripW;  // strip width
    __shared__ S ring1[9][RING + 2][SW + 4];
    __shared__ S ring2[9][RING + 2][NARROW ? SW + 3 : SW + 2];
    __shared__ int s_skip;
    const int tid = threadIdx.x;
    const unsigned xcc = xcc_id();
    unsigned rank, count;
    long long n0;
    if (!register_group(bar, xtab, err, timeout_ticks, xcc, step_ctr, rank, count, n0)) return;
    const int first_strip = xtab[2 * xcc], nstrips = xtab[2 * xcc + 1];
    unsigned* xbar = bar + kLine * (1 + kMaxXcc + xcc);
    for (int p = 0; p < ntriples; ++p) {
        const long long n = n0 + (advance ? 3 * p : 0);
        const int sc = (int)(n0 & 1) ^ (advance ? (p & 1) : 0);
        const S* src = base + sc * copy_elems;
        S* dst = base + (sc ^ 1) * copy_elems;
        for (int t = (int)rank; t < nstrips; t += (int)count) {
            const int2 e = run[first_strip + t];  // (instance, strip within the instance)
            const int j = e.x;
            const BDesc<R>& d = desc[j];
            if (tid == 0) {
                const int frozen = __hip_atomic_load(blowup + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_skip = ((long long)frozen < n || !active[j]) ? 1 : 0;  // blew up earlier, or retired
                if (!s_skip && advance && e.y == 0) lastcopy[j] = sc ^ 1;
            }
            __syncthreads();
            const bool skip = s_skip != 0;
            __syncthreads();  // s_skip is rewritten for the next strip only after every thread read it
            if (skip) continue;
            const int gsx = (d.nx + SW - 1) / SW;
            const int sy = e.y / gsx;
            const int x0 = (e.y - sy * gsx) * SW, ys = sy * hs;
            const Geom g{d.nx, d.ny, d.plane};
            auto coll = [&](R(&h)[9], const Macro<R>& m) { collide_model(d.model, h, m, d.ref, d.c, d.N); };
            if constexpr (NARROW)
                strip_three_steps_narrow<RING, SW, true, false>(ring1, ring2, src + d.off, dst + d.off, g, d.ref, x0, ys,
                                                                min(ys + hs, d.ny), (int)n, blowup + j, coll);
            else
                strip_three_steps<RING, kStripW, true, false>(ring1, ring2, src + d.off, dst + d.off, g, d.ref, x0, ys,
                                                              min(ys + hs, d.ny), (int)n, blowup + j, coll);
        }
        if (!xcd_barrier(xbar, p, count, err, timeout_ticks)) return;
    }
    if (advance && blockIdx.x == 0 && tid == 0) *step_ctr = n0 + 3LL * ntriples;
}

// XCD of each workgroup of a small probe launch (which XCC ids the device dispatches to).
__global__ void k_xcc_probe(int* __restrict__ out) {
    if (threadIdx.x == 0) out[blockIdx.x] = (int)xcc_id();
}

// f(., 0) = f^eq of every instance, stored pre-streamed into copy 0.  One block per tile of
// the NPT = 1 table.
template <int PREC>
__global__ __launch_bounds__(kTileThreads) void k_batch_init(
    typename Store<PREC>::S* __restrict__ base, const BDesc<typename Store<PREC>::R>* __restrict__ desc,
    const int* __restrict__ tile_inst, const double* __restrict__ rho, const double* __restrict__ ux,
    const double* __restrict__ uy) {
    const int j = tile_inst[blockIdx.x];
    const BDesc<typename Store<PREC>::R>& d = desc[j];
    const int c = (blockIdx.x - d.tile0) * kTileThreads + threadIdx.x;
    if (c >= d.cells) return;
    const int y = row_of(c, d.nx, d.inv_nx);
    const int x = c - y * d.nx;
    double h[9];
    eq_deviation(rho[d.foff + c], ux[d.foff + c], uy[d.foff + c], d.ref_d, d.N, h);
    prestream_store(base + d.off, Geom{d.nx, d.ny, d.plane}, x, y, h);
}

template <int PREC>
__global__ __launch_bounds__(256) void k_batch_get(const typename Store<PREC>::S* __restrict__ src,
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

// Mean of |u|^2 over the nodes of every instance (FP64, pulled from the copy of the current
// step): one block per 256-node tile writes its partial sum, then one thread per instance adds
// its tiles in order (deterministic).
template <int PREC>
__global__ __launch_bounds__(kTileThreads) void k_batch_u2_tiles(
    const typename Store<PREC>::S* __restrict__ base, long long copy_elems, const long long* __restrict__ step_ctr,
    const BDesc<typename Store<PREC>::R>* __restrict__ desc, const int* __restrict__ tile_inst,
    double* __restrict__ partial) {
    __shared__ double red[kTileThreads / 64];
    // the copy of the current step's parity (read on the device: a replayed graph advances the
    // counter without the host)
    const typename Store<PREC>::S* cur = base + (*step_ctr & 1) * copy_elems;
    const int j = tile_inst[blockIdx.x];
    const BDesc<typename Store<PREC>::R>& d = desc[j];
    const int c = (blockIdx.x - d.tile0) * kTileThreads + threadIdx.x;
    double v = 0.0;
    if (c < d.cells) {
        const int y = row_of(c, d.nx, d.inv_nx);
        const int x = c - y * d.nx;
        const Nbr nb = neighbours(x, y, d.nx, d.ny);
        double h[9];
        pull_load(cur + d.off, d.plane, nb, h);
        const Ref<double>& r = d.ref_d;
        const double rho = r.rho + (((h[0] + (h[1] + h[3])) + (h[2] + h[4])) + ((h[5] + h[7]) + (h[6] + h[8])));
        const double jx = ((h[1] + h[5] + h[8]) - (h[3] + h[6] + h[7])) + r.rho * r.ux;
        const double jy = ((h[2] + h[5] + h[6]) - (h[4] + h[7] + h[8])) + r.rho * r.uy;
        const double ux = jx / rho, uy = jy / rho;
        v = ux * ux + uy * uy;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename R>
__global__ void k_batch_u2_sum(const BDesc<R>* __restrict__ desc, int n, const double* __restrict__ partial,
                               double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const BDesc<R>& d = desc[j];
    const int nt = (d.cells + kTileThreads - 1) / kTileThreads;
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += partial[d.tile0 + t];
    out[j] = s / (double)d.cells;
}

// Retire the instances whose flag is 0 (for good) and record the step at which they left.
__global__ void k_retire(const int* __restrict__ flags, int* __restrict__ active, int* __restrict__ retired,
                         int n, const long long* __restrict__ step_ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && active[i] && !flags[i]) {
        active[i] = 0;
        retired[i] = (int)*step_ctr;
    }
}

// Reset the barrier counter before each replay.  The error flag is sticky (cleared only at
// creation) so that a stopped launch stays reported.
__global__ void k_batch_reset(unsigned* __restrict__ bar) {
    for (int i = threadIdx.x; i < kBarrierWords; i += blockDim.x) bar[i] = 0u;
}

__global__ void k_clear_i32(int* __restrict__ p) {
    if (threadIdx.x == 0) *p = 0;
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

struct lbm_batch {
    int n = 0, prec = 0;
    std::vector<lbm_instance_desc> hdesc;
    std::vector<long long> off, plane, foff;
    long long copy_elems = 0;
    char* buf = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;      // caller's stream
    // launch shapes k: 0, 1, 2 = one step per pass with 1, 2, 4 nodes per thread; 3 = two
    // steps per pass over strips; 4 = three steps per pass over the same strips (shape 3's run
    // table)
    int cus = 0, occ[5] = {0, 0, 0, 0, 0};     // CUs, occupancy limit per shape (runtime query)
    int res_fit[5] = {0, 0, 0, 0, 0};          // groups per CU the kernel's own resources allow
    int resident[5] = {0, 0, 0, 0, 0};         // groups per CU confirmed co-resident (0 = not probed)
    int npt = 1, gpc = 0;              // launch shape (gpc 0 = occupancy limit)
    // fused passes over strips of hs rows (64: on the 512-instance FP64 sweep with three steps per
    // pass on 48-column strips 77-78 GLUPS against 75 with 32 rows, 69 with 16, 76-77 with 80-128)
    int fuse = 0, hs = 64;
    int depth = 2;                     // steps per fused pass: 2 (runs of 4 steps) or 3
    long long step = 0;                // host mirror of the step counter
    void* d_desc[3] = {nullptr, nullptr, nullptr};  // descriptors per NPT (tile0 differs)
    int* d_tiles[3] = {nullptr, nullptr, nullptr};  // every tile of every instance, instance order
    int ntiles[3] = {0, 0, 0};
    // tiles / strips of live instances per launch shape, one list per XCD (shape 4: the strips of the
    // three-step kernel, 48 columns wide in FP64)
    int2* d_run[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int* d_xtab[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per XCC id: first run entry, entry count
    long long run_cap[5] = {0, 0, 0, 0, 0};                          // entries d_run[k] can hold
    std::vector<int> xccs;                          // XCC ids the device dispatches to
    int* d_blowup = nullptr;
    int* d_active = nullptr;           // per instance: nonzero = advanced by lbm_batch_run
    int* d_retired = nullptr;          // per instance: step at which it was retired (INT_MAX)
    int* d_lastcopy = nullptr;         // per instance: copy its last pass wrote (0 before any)
    double* d_u2part = nullptr;        // per 256-node tile: partial sums of |u|^2
    unsigned* d_bar = nullptr;
    int* d_err = nullptr;
    long long* d_step = nullptr;
    long long timeout_ticks = 0;
    long long probe_ticks = 0;
    int probe_stepdowns = 0;           // residency probes that had to lower a shape's groups per CU
};

namespace {

int npt_index(int npt) { return npt == 4 ? 2 : (npt == 2 ? 1 : 0); }

template <int PREC>
const void* batch_kernel(int npt) {
    switch (npt) {
        case 4: return batch1_fn<PREC, 4>();
        case 2: return batch1_fn<PREC, 2>();
        default: return batch1_fn<PREC, 1>();
    }
}

const void* batch_kernel_p(int prec, int npt) {
    switch (prec) {
        case LBM_F64: return batch_kernel<kF64>(npt);
        case LBM_F32_SHIFTED: return batch_kernel<kF32>(npt);
        default: return batch_kernel<kF16>(npt);
    }
}

// The persistent kernel is launched cooperatively, at a grid size from its resources
// (resources_fit) that all CUs hold at once.  The runtime's own check of a cooperative launch uses
// its occupancy figure, which can be larger than what is resident (see sgpr_waves), so it does not
// replace that sizing; the bounded barrier waits are the safety net.
template <int PREC, int NPT>
hipError_t launch_batch_t(lbm_batch* b, hipStream_t s, int G, int nsteps, int advance) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    const int k = npt_index(NPT);
    S* base = reinterpret_cast<S*>(b->buf);
    long long copy_elems = b->copy_elems;
    const BDesc<R>* desc = reinterpret_cast<const BDesc<R>*>(b->d_desc[k]);
    const int2* tiles = b->d_run[k];
    const int* xtab = b->d_xtab[k];
    int* blowup = b->d_blowup;
    const int* active = b->d_active;
    int* lastcopy = b->d_lastcopy;
    unsigned* bar = b->d_bar;
    int* err = b->d_err;
    long long* step = b->d_step;
    long long timeout = b->timeout_ticks;
    void* args[] = {&base, &copy_elems, &desc, &tiles, &xtab, &blowup, &active, &lastcopy, &bar, &err, &step,
                    &nsteps, &advance, &timeout};
    return hipLaunchCooperativeKernel(batch1_fn<PREC, NPT>(), dim3(G),
                                      dim3(kTileThreads), args, 0, s);
}

constexpr int kBatchRing = 8;

template <int PREC>
hipError_t launch_batch2_t(lbm_batch* b, hipStream_t s, int G, int npairs, int advance) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    S* base = reinterpret_cast<S*>(b->buf);
    long long copy_elems = b->copy_elems;
    const BDesc<R>* desc = reinterpret_cast<const BDesc<R>*>(b->d_desc[0]);
    const int2* strips = b->d_run[3];
    const int* xtab = b->d_xtab[3];
    int* blowup = b->d_blowup;
    const int* active = b->d_active;
    int* lastcopy = b->d_lastcopy;
    unsigned* bar = b->d_bar;
    int* err = b->d_err;
    long long* step = b->d_step;
    long long timeout = b->timeout_ticks;
    int hs = b->hs;
    void* args[] = {&base, &copy_elems, &desc, &strips, &xtab, &blowup, &active, &lastcopy, &bar, &err, &step,
                    &npairs, &advance, &timeout, &hs};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch2<PREC, kBatchRing>), dim3(G),
                                      dim3(kTileThreads), args, 0, s);
}

const void* batch2_kernel_p(int prec) {
    switch (prec) {
        case LBM_F64: return reinterpret_cast<const void*>(&k_batch2<kF64, kBatchRing>);
        case LBM_F32_SHIFTED: return reinterpret_cast<const void*>(&k_batch2<kF32, kBatchRing>);
        default: return reinterpret_cast<const void*>(&k_batch2<kF16, kBatchRing>);
    }
}

constexpr int kBatch3Ring = 4;

template <int PREC>
hipError_t launch_batch3_t(lbm_batch* b, hipStream_t s, int G, int ntriples, int advance) {
    using S = typename Store<PREC>::S;
    using R = typename Store<PREC>::R;
    S* base = reinterpret_cast<S*>(b->buf);
    long long copy_elems = b->copy_elems;
    const BDesc<R>* desc = reinterpret_cast<const BDesc<R>*>(b->d_desc[0]);
    const int2* strips = b->d_run[4];
    const int* xtab = b->d_xtab[4];
    int* blowup = b->d_blowup;
    const int* active = b->d_active;
    int* lastcopy = b->d_lastcopy;
    unsigned* bar = b->d_bar;
    int* err = b->d_err;
    long long* step = b->d_step;
    long long timeout = b->timeout_ticks;
    int hs = b->hs;
    void* args[] = {&base, &copy_elems, &desc, &strips, &xtab, &blowup, &active, &lastcopy, &bar, &err, &step,
                    &ntriples, &advance, &timeout, &hs};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch3<PREC, kBatch3Ring>), dim3(G),
                                      dim3(kTileThreads), args, 0, s);
}

// The three-step kernel exists for FP64 and FP32 (nullptr for FP16).
const void* batch3_kernel_p(int prec) {
    switch (prec) {
        case LBM_F64: return reinterpret_cast<const void*>(&k_batch3<kF64, kBatch3Ring>);
        case LBM_F32_SHIFTED: return reinterpret_cast<const void*>(&k_batch3<kF32, kBatch3Ring>);
        default: return nullptr;
    }
}

long long strips_of(const lbm_instance_desc& d, int hs, int width = kStripW) {
    return (long long)((d.nx + width - 1) / width) * ((d.ny + hs - 1) / hs);
}

// Strip width of the three-step batched kernel (launch shape 4).
int batch3_width(int prec) { return prec == LBM_F64 ? kBatchNarrowW : kStripW; }

template <int PREC>
hipError_t launch_batch_p(lbm_batch* b, hipStream_t s, int G, int nsteps, int advance) {
    switch (b->npt) {
        case 4: return launch_batch_t<PREC, 4>(b, s, G, nsteps, advance);
        case 2: return launch_batch_t<PREC, 2>(b, s, G, nsteps, advance);
        default: return launch_batch_t<PREC, 1>(b, s, G, nsteps, advance);
    }
}

// Deal the live instances to the XCDs, largest first, each to the XCD with the fewest nodes so
// far, and write each launch shape's run table (one contiguous list of (instance, tile) per XCD,
// instances in index order within it) and XCD table.  Synchronous.
int deal_tables(lbm_batch* b, const std::vector<char>& live) {
    const int n = b->n;
    std::vector<int> order;
    for (int j = 0; j < n; ++j)
        if (live[j]) order.push_back(j);
    auto cells = [&](int j) { return (long long)b->hdesc[j].nx * b->hdesc[j].ny; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cells(a) > cells(c); });
    std::vector<long long> load(b->xccs.size(), 0);
    std::vector<int> owner((size_t)n, -1);
    for (int j : order) {
        size_t best = 0;
        for (size_t q = 1; q < b->xccs.size(); ++q)
            if (load[q] < load[best]) best = q;
        load[best] += cells(j);
        owner[j] = b->xccs[best];
    }
    const int npts[3] = {1, 2, 4};
    for (int k = 0; k < 5; ++k) {
        if (k == 4 && !b->d_run[4]) continue;  // no three-step kernel (FP16)
        std::vector<int2> run;
        std::vector<int> xtab(2 * kMaxXcc, 0);
        for (int x : b->xccs) {
            xtab[2 * x] = (int)run.size();
            for (int j = 0; j < n; ++j) {
                if (owner[j] != x) continue;
                const long long nt = k < 3 ? (cells(j) + (long long)kTileThreads * npts[k] - 1) /
                                                 ((long long)kTileThreads * npts[k])
                                           : strips_of(b->hdesc[j], b->hs, k == 4 ? batch3_width(b->prec) : kStripW);
                for (int t = 0; t < (int)nt; ++t) run.push_back(make_int2(j, t));
            }
            xtab[2 * x + 1] = (int)run.size() - xtab[2 * x];
        }
        if ((long long)run.size() > b->run_cap[k]) return set_error(LBM_EHIP, "run table %d overflow", k);
        int rc = LBM_OK;
        if (!run.empty())
            rc = check_hip(hipMemcpy(b->d_run[k], run.data(), sizeof(int2) * run.size(), hipMemcpyHostToDevice),
                           "copy run table");
        if (rc == LBM_OK)
            rc = check_hip(hipMemcpy(b->d_xtab[k], xtab.data(), sizeof(int) * xtab.size(), hipMemcpyHostToDevice),
                           "copy xtab");
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

int shape_of(const lbm_batch* b, bool fused) { return fused ? (b->depth == 3 ? 4 : 3) : npt_index(b->npt); }

// Workgroups of `threads` threads that one CU holds at once for kernel fn, from the kernel's own
// resources and the CU's: every SIMD (four per CU) has 512 VGPRs per lane, allocated in granules of
// 8, at most 8 waves, and room for the waves that sgpr_waves gives for the kernel's SGPR bound; a
// workgroup's waves are spread over the SIMDs; the CU's LDS and thread slots are shared by its
// workgroups.
int resources_fit(const void* fn, int threads, int sgprs, int* out) {
    hipFuncAttributes a{};
    int dev = 0, lds_cu = 0, thr_cu = 0;
    int rc = check_hip(hipFuncGetAttributes(&a, fn), "hipFuncGetAttributes");
    if (rc == LBM_OK) rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc == LBM_OK)
        rc = check_hip(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev),
                       "LDS per CU");
    if (rc == LBM_OK)
        rc = check_hip(hipDeviceGetAttribute(&thr_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev),
                       "threads per CU");
    if (rc != LBM_OK) return rc;
    const int waves = (threads + 63) / 64;
    const int vgpr = std::max(8, (a.numRegs + 7) / 8 * 8);
    const int waves_per_simd = std::min(std::min(8, 512 / vgpr), sgpr_waves(sgprs));
    int fit = waves_per_simd * 4 / waves;
    if (a.sharedSizeBytes > 0) fit = std::min(fit, lds_cu / (int)a.sharedSizeBytes);
    if (thr_cu > 0) fit = std::min(fit, thr_cu / threads);
    *out = fit;
    return fit >= 1 ? LBM_OK : set_error(LBM_EHIP, "persistent kernel does not fit a CU");
}

// Groups per CU of a launch of shape k: the probed figure once known, else the smaller of the
// kernel's resource figure and the runtime's occupancy query.
int groups_limit(lbm_batch* b, int k) {
    if (b->resident[k] > 0) return b->resident[k];
    return b->res_fit[k] > 0 ? std::min(b->res_fit[k], b->occ[k]) : b->occ[k];
}

int grid_size(lbm_batch* b, int k) {
    const int lim = groups_limit(b, k);
    const int per = (b->gpc <= 0 || b->gpc > lim) ? lim : b->gpc;
    return b->cus * per;
}

// Reset the barrier counter, then one cooperative launch of the persistent kernel of shape k on
// G groups: `units` steps (shapes 0-2), pairs of steps (shape 3) or triples (shape 4).
int run_persistent_on(lbm_batch* b, int k, int G, int units, int advance, long long ticks) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, b->d_bar);
    int rc = check_hip(hipGetLastError(), "barrier reset launch");
    if (rc != LBM_OK) return rc;
    const long long keep = b->timeout_ticks;
    b->timeout_ticks = ticks;
    hipError_t e;
    if (k == 4) {
        switch (b->prec) {
            case LBM_F64: e = launch_batch3_t<kF64>(b, b->stream, G, units, advance); break;
            case LBM_F32_SHIFTED: e = launch_batch3_t<kF32>(b, b->stream, G, units, advance); break;
            default: e = hipErrorInvalidValue; break;
        }
    } else if (k == 3) {
        switch (b->prec) {
            case LBM_F64: e = launch_batch2_t<kF64>(b, b->stream, G, units, advance); break;
            case LBM_F32_SHIFTED: e = launch_batch2_t<kF32>(b, b->stream, G, units, advance); break;
            default: e = launch_batch2_t<kF16>(b, b->stream, G, units, advance); break;
        }
    } else {
        switch (b->prec) {
            case LBM_F64: e = launch_batch_p<kF64>(b, b->stream, G, units, advance); break;
            case LBM_F32_SHIFTED: e = launch_batch_p<kF32>(b, b->stream, G, units, advance); break;
            default: e = launch_batch_p<kF16>(b, b->stream, G, units, advance); break;
        }
    }
    b->timeout_ticks = keep;
    return check_hip(e, "cooperative launch of the persistent kernel");
}

int run_persistent(lbm_batch* b, int k, int units, int advance) {
    return run_persistent_on(b, k, grid_size(b, k), units, advance, b->timeout_ticks);
}

// A persistent grid larger than what the CUs hold at once cannot pass its first barrier.  The
// grid is sized from the kernel's own resources (resources_fit, no larger than the runtime's
// occupancy query).  As a safety net, before the first run of each launch shape a probe runs two
// non-advancing steps (or pairs or triples; they recompute from the same copy: state, counters and
// records unchanged) with a short barrier bound, and steps the figure down only if that grid did
// not pass every barrier (counted in probe_stepdowns).  A failed probe ends by its bound: every
// wave exits.
int ensure_resident(lbm_batch* b, int k) {
    if (b->resident[k] > 0) return LBM_OK;
    for (int per = groups_limit(b, k); per >= 1; --per) {
        int rc = run_persistent_on(b, k, b->cus * per, 2, 0, b->probe_ticks);
        if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(b->stream), "synchronise (residency probe)");
        int err = 0;
        if (rc == LBM_OK) rc = check_hip(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost), "copy err");
        if (rc != LBM_OK) return rc;
        if (!err) {
            b->resident[k] = per;
            return LBM_OK;
        }
        ++b->probe_stepdowns;
        if (err == 2) return set_error(LBM_EHIP, "an XCD that owns instances got no workgroup");
        hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, b->stream, b->d_err);
        rc = check_hip(hipGetLastError(), "clear err");
        if (rc != LBM_OK) return rc;
    }
    return set_error(LBM_EHIP, "no persistent grid of this shape stays co-resident");
}

// Advance every live instance by `units` steps (k < 3), pairs (k = 3) or triples (k = 4), in
// launches short enough that the barrier counter G * units stays below 2^31.
int run_units(lbm_batch* b, int k, int units) {
    if (units <= 0) return LBM_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    int rc = check_hip(hipStreamIsCapturing(b->stream, &cap), "hipStreamIsCapturing");
    if (rc != LBM_OK) return rc;
    const bool capturing = cap != hipStreamCaptureStatusNone;
    // the residency probe synchronises: it cannot run inside a stream capture
    if (capturing && b->resident[k] == 0)
        return set_error(LBM_ESTATE, "launch shape not probed yet: run (or autotune) the batch once with the "
                                     "same settings before capturing it");
    rc = ensure_resident(b, k);
    if (rc != LBM_OK) return rc;
    const long long G = grid_size(b, k);
    const int chunk = (int)std::min<long long>(units, (1LL << 31) / G);
    int left = units;
    while (left > 0) {
        const int u = std::min(left, chunk);
        rc = run_persistent(b, k, u, 1);
        if (rc != LBM_OK) return rc;
        left -= u;
        // a captured launch runs only when the graph is replayed; the synchronising calls then
        // take the step from the device counter
        if (!capturing) b->step += k == 4 ? 3LL * u : (k == 3 ? 2LL * u : (long long)u);
    }
    return LBM_OK;
}

// Live instances: neither blown up nor retired.  Synchronous.
int live_set(lbm_batch* b, std::vector<char>& live) {
    std::vector<int> blow((size_t)b->n), ret((size_t)b->n);
    int rc = check_hip(hipStreamSynchronize(b->stream), "synchronise");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(blow.data(), b->d_blowup, sizeof(int) * blow.size(), hipMemcpyDeviceToHost),
                       "copy blow-up steps");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(ret.data(), b->d_retired, sizeof(int) * ret.size(), hipMemcpyDeviceToHost),
                       "copy retired steps");
    if (rc != LBM_OK) return rc;
    live.assign((size_t)b->n, 0);
    for (int j = 0; j < b->n; ++j) live[j] = blow[j] == INT_MAX && ret[j] == INT_MAX;
    return LBM_OK;
}

// (Re)allocate strip table k to hold `total` strips.
int alloc_table(lbm_batch* b, int k, long long total) {
    if (total >= INT_MAX) return set_error(LBM_EINVAL, "too many strips (%lld)", total);
    if (b->d_run[k] && total <= b->run_cap[k]) return LBM_OK;
    if (b->d_run[k]) (void)hipFree(b->d_run[k]);
    b->d_run[k] = nullptr;
    b->run_cap[k] = 0;
    int rc = check_hip(hipMalloc(&b->d_run[k], sizeof(int2) * (size_t)std::max(1LL, total)), "hipMalloc(strip run)");
    if (rc == LBM_OK) b->run_cap[k] = total;
    return rc;
}

// (Re)allocate the strip tables (two and three steps per pass) for the current strip height.
int alloc_strips(lbm_batch* b) {
    long long t3 = 0, t4 = 0;
    for (int j = 0; j < b->n; ++j) {
        t3 += strips_of(b->hdesc[j], b->hs);
        t4 += strips_of(b->hdesc[j], b->hs, batch3_width(b->prec));
    }
    int rc = alloc_table(b, 3, t3);
    if (rc == LBM_OK && batch3_kernel_p(b->prec)) rc = alloc_table(b, 4, t4);
    return rc;
}

}  // namespace

extern "C" {

size_t lbm_batch_population_bytes(const lbm_instance_desc* desc, int n, int prec) {
    if (!desc || n < 1 || prec < LBM_F64 || prec > LBM_F16_SHIFTED) return 0;
    long long total = 0;
    for (int j = 0; j < n; ++j) {
        if (desc[j].nx < 2 || desc[j].ny < 2 || (long long)desc[j].nx * desc[j].ny >= (1LL << 24)) return 0;
        total += 9 * plane_elems(desc[j].nx, desc[j].ny, prec);
    }
    if (2 * total >= (1LL << 40)) return 0;
    return (size_t)(2 * total * (long long)elem_size(prec));
}

int lbm_batch_create(lbm_batch** out, const lbm_instance_desc* desc, int n, int prec,
                     const double* rho, const double* ux, const double* uy, void* pop_buf,
                     size_t pop_bytes, void* hip_stream) {
    if (!out) return set_error(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc || n < 1) return set_error(LBM_EINVAL, "need n >= 1 descriptors");
    if (prec < LBM_F64 || prec > LBM_F16_SHIFTED) return set_error(LBM_EINVAL, "unknown precision %d", prec);
    for (int j = 0; j < n; ++j) {
        const lbm_instance_desc& d = desc[j];
        if (d.nx < 2 || d.ny < 2 || (long long)d.nx * d.ny >= (1LL << 24))
            return set_error(LBM_EINVAL, "instance %d: grid %d x %d out of range", j, d.nx, d.ny);
        if (d.model < LBM_BGK || d.model > LBM_RR)
            return set_error(LBM_EINVAL, "instance %d: model %d not a collision model", j, d.model);
        if (d.eq_order < 2 || d.eq_order > 4)
            return set_error(LBM_EINVAL, "instance %d: eq_order %d", j, d.eq_order);
        int rc = validate_model(d.model, d.eq_order);
        if (rc == LBM_OK) rc = validate_omega(d.omega);
        if (rc != LBM_OK) return rc;
        if (prec != LBM_F64 && !(d.rho0 > 0.0))
            return set_error(LBM_EINVAL, "instance %d: rho0 must be > 0", j);
        if (prec != LBM_F64 && !(d.ux0 * d.ux0 + d.uy0 * d.uy0 < 1.0))
            return set_error(LBM_EINVAL, "instance %d: reference velocity must have |U| < 1", j);
    }
    if (!rho || !ux || !uy || !pop_buf) return set_error(LBM_EINVAL, "NULL device pointer");
    if (reinterpret_cast<uintptr_t>(pop_buf) % 256 != 0)
        return set_error(LBM_EINVAL, "pop_buf must be 256-byte aligned");
    const size_t need = lbm_batch_population_bytes(desc, n, prec);
    if (need == 0 || pop_bytes < need)
        return set_error(LBM_EINVAL, "pop_bytes %zu < required %zu", pop_bytes, need);

    lbm_batch* b = new lbm_batch();
    b->n = n;
    b->prec = prec;
    b->hdesc.assign(desc, desc + n);
    b->buf = static_cast<char*>(pop_buf);
    b->bytes = pop_bytes;
    b->stream = static_cast<hipStream_t>(hip_stream);
    long long o = 0, fo = 0;
    for (int j = 0; j < n; ++j) {
        const long long pl = plane_elems(desc[j].nx, desc[j].ny, prec);
        b->off.push_back(o);
        b->plane.push_back(pl);
        b->foff.push_back(fo);
        o += 9 * pl;
        fo += (long long)desc[j].nx * desc[j].ny;
    }
    b->copy_elems = o;

    int rc = LBM_OK;
    int dev = 0, clock_khz = 0;
    rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc == LBM_OK) rc = check_hip(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (rc == LBM_OK) rc = check_hip(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
    b->timeout_ticks = 2LL * 1000LL * (long long)(clock_khz > 0 ? clock_khz : 100000);  // 2 s
    b->probe_ticks = b->timeout_ticks / 8;                                                // 250 ms
    int coop = 0;
    if (rc == LBM_OK) rc = check_hip(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev), "cooperative launch attribute");
    if (rc == LBM_OK && !coop) rc = set_error(LBM_EUNSUPPORTED, "device does not support cooperative launches");
    // which XCC ids the device dispatches to (the instances are dealt to them below)
    std::vector<int>& xccs = b->xccs;
    if (rc == LBM_OK) {
        const int nprobe = 4 * b->cus;
        int* d_probe = nullptr;
        std::vector<int> seen((size_t)nprobe, 0);
        rc = check_hip(hipMalloc(&d_probe, sizeof(int) * (size_t)nprobe), "hipMalloc(xcc probe)");
        if (rc == LBM_OK) {
            hipLaunchKernelGGL(k_xcc_probe, dim3(nprobe), dim3(64), 0, b->stream, d_probe);
            rc = check_hip(hipGetLastError(), "xcc probe launch");
        }
        if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(b->stream), "synchronise (xcc probe)");
        if (rc == LBM_OK)
            rc = check_hip(hipMemcpy(seen.data(), d_probe, sizeof(int) * seen.size(), hipMemcpyDeviceToHost),
                           "copy xcc probe");
        if (d_probe) (void)hipFree(d_probe);
        bool have[kMaxXcc] = {};
        for (int v : seen) have[v & (kMaxXcc - 1)] = true;
        for (int x = 0; x < kMaxXcc; ++x)
            if (have[x]) xccs.push_back(x);
    }
    if (rc == LBM_OK && xccs.empty()) rc = set_error(LBM_EHIP, "no XCD seen by the probe launch");
    const int npts[3] = {1, 2, 4};
    for (int k = 0; k < 3 && rc == LBM_OK; ++k) {
        rc = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[k], batch_kernel_p(prec, npts[k]),
                                                                    kTileThreads, 0),
                       "occupancy");
        if (rc == LBM_OK && b->occ[k] < 1) rc = set_error(LBM_EHIP, "persistent kernel does not fit a CU");
        if (rc == LBM_OK)
            rc = resources_fit(batch_kernel_p(prec, npts[k]), kTileThreads, prec == LBM_F64 ? batch1_sgprs<kF64>() :
                               batch1_sgprs<kF32>(), &b->res_fit[k]);
        // tile table and descriptors for this NPT
        const int tile_nodes = kTileThreads * npts[k];
        std::vector<int> tiles, tile0((size_t)n, 0);
        for (int j = 0; j < n; ++j) {
            const int cells = desc[j].nx * desc[j].ny;
            tile0[j] = (int)tiles.size();
            for (int t = 0; t < (cells + tile_nodes - 1) / tile_nodes; ++t) tiles.push_back(j);
        }
        std::vector<char> dbytes;
        const size_t dsz = prec == LBM_F64 ? sizeof(BDesc<double>) : sizeof(BDesc<float>);
        dbytes.resize(dsz * (size_t)n);
        for (int j = 0; j < n && rc == LBM_OK; ++j) {
            const lbm_instance_desc& d = desc[j];
            const int cells = d.nx * d.ny;
            const int t0 = tile0[j];
            const Ref<double> rd = storage_reference(prec, d.rho0, d.ux0, d.uy0);
            if (prec == LBM_F64) {
                BDesc<double> bd;
                bd.nx = d.nx; bd.ny = d.ny; bd.model = d.model; bd.N = d.eq_order;
                bd.cells = cells; bd.tile0 = t0; bd.off = b->off[j]; bd.plane = b->plane[j];
                bd.foff = b->foff[j]; bd.inv_nx = 1.0f / (float)d.nx;
                bd.ref = ref_as<double>(rd); bd.ref_d = rd;
                bd.c = make_coef<double>(d.omega);
                std::memcpy(dbytes.data() + dsz * j, &bd, dsz);
            } else {
                BDesc<float> bd;
                bd.nx = d.nx; bd.ny = d.ny; bd.model = d.model; bd.N = d.eq_order;
                bd.cells = cells; bd.tile0 = t0; bd.off = b->off[j]; bd.plane = b->plane[j];
                bd.foff = b->foff[j]; bd.inv_nx = 1.0f / (float)d.nx;
                bd.ref = ref_as<float>(rd); bd.ref_d = rd;
                bd.c = make_coef<float>(d.omega);
                std::memcpy(dbytes.data() + dsz * j, &bd, dsz);
            }
        }
        b->ntiles[k] = (int)tiles.size();
        if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_desc[k], dbytes.size()), "hipMalloc(desc)");
        if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_tiles[k], sizeof(int) * tiles.size()), "hipMalloc(tiles)");
        if (rc == LBM_OK)
            rc = check_hip(hipMemcpy(b->d_desc[k], dbytes.data(), dbytes.size(), hipMemcpyHostToDevice), "copy desc");
        if (rc == LBM_OK)
            rc = check_hip(hipMemcpy(b->d_tiles[k], tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice),
                           "copy tiles");
        if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_run[k], sizeof(int2) * tiles.size()), "hipMalloc(run)");
        if (rc == LBM_OK) b->run_cap[k] = (long long)tiles.size();
        if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_xtab[k], sizeof(int) * 2 * kMaxXcc), "hipMalloc(xtab)");
    }
    // two steps per pass: occupancy, strip table
    if (rc == LBM_OK)
        rc = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[3], batch2_kernel_p(prec), kTileThreads, 0),
                       "occupancy");
    if (rc == LBM_OK && b->occ[3] < 1) rc = set_error(LBM_EHIP, "persistent two-step kernel does not fit a CU");
    if (rc == LBM_OK) rc = resources_fit(batch2_kernel_p(prec), kTileThreads, kBatchFusedSgprs, &b->res_fit[3]);
    if (rc == LBM_OK && batch3_kernel_p(prec))
        rc = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->occ[4], batch3_kernel_p(prec), kTileThreads, 0),
                       "occupancy");
    if (rc == LBM_OK && batch3_kernel_p(prec) && b->occ[4] < 1)
        rc = set_error(LBM_EHIP, "persistent three-step kernel does not fit a CU");
    if (rc == LBM_OK && batch3_kernel_p(prec))
        rc = resources_fit(batch3_kernel_p(prec), kTileThreads, kBatchFusedSgprs, &b->res_fit[4]);
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_xtab[3], sizeof(int) * 2 * kMaxXcc), "hipMalloc(xtab)");
    if (rc == LBM_OK && batch3_kernel_p(prec))
        rc = check_hip(hipMalloc(&b->d_xtab[4], sizeof(int) * 2 * kMaxXcc), "hipMalloc(xtab)");
    if (rc == LBM_OK) rc = alloc_strips(b);
    if (rc == LBM_OK) rc = deal_tables(b, std::vector<char>((size_t)n, 1));
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_blowup, sizeof(int) * (size_t)n), "hipMalloc(blowup)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_active, sizeof(int) * (size_t)n), "hipMalloc(active)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_retired, sizeof(int) * (size_t)n), "hipMalloc(retired)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_lastcopy, sizeof(int) * (size_t)n), "hipMalloc(lastcopy)");
    if (rc == LBM_OK)
        rc = check_hip(hipMalloc(&b->d_u2part, sizeof(double) * (size_t)b->ntiles[0]), "hipMalloc(u2 partials)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_bar, sizeof(unsigned) * kBarrierWords), "hipMalloc(barrier)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_err, sizeof(int)), "hipMalloc(err)");
    if (rc == LBM_OK) rc = check_hip(hipMalloc(&b->d_step, sizeof(long long)), "hipMalloc(step)");
    if (rc == LBM_OK) {
        const long long zero = 0;
        rc = check_hip(hipMemcpy(b->d_step, &zero, sizeof(zero), hipMemcpyHostToDevice), "reset step");
    }
    if (rc == LBM_OK) {
        hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->d_blowup, n, INT_MAX);
        hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->d_active, n, 1);
        hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->d_retired, n, INT_MAX);
        hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->d_lastcopy, n, 0);
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, b->d_bar);
        hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, b->stream, b->d_err);
        switch (prec) {
            case LBM_F64:
                hipLaunchKernelGGL(k_batch_init<kF64>, dim3(b->ntiles[0]), dim3(kTileThreads), 0, b->stream,
                                   reinterpret_cast<double*>(b->buf),
                                   reinterpret_cast<const BDesc<double>*>(b->d_desc[0]), b->d_tiles[0], rho, ux, uy);
                break;
            case LBM_F32_SHIFTED:
                hipLaunchKernelGGL(k_batch_init<kF32>, dim3(b->ntiles[0]), dim3(kTileThreads), 0, b->stream,
                                   reinterpret_cast<float*>(b->buf),
                                   reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->d_tiles[0], rho, ux, uy);
                break;
            default:
                hipLaunchKernelGGL(k_batch_init<kF16>, dim3(b->ntiles[0]), dim3(kTileThreads), 0, b->stream,
                                   reinterpret_cast<_Float16*>(b->buf),
                                   reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->d_tiles[0], rho, ux, uy);
                break;
        }
        rc = check_hip(hipGetLastError(), "batch init launch");
    }
    if (rc != LBM_OK) {
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_run(lbm_batch* b, int nsteps) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps %d < 0", nsteps);
    if (b->step + nsteps >= INT_MAX) return set_error(LBM_EINVAL, "step counter would overflow");
    if (nsteps == 0) return LBM_OK;
    // three steps per pass (any number of triples leaves every live state in the copy of its
    // step's parity), or two in runs of 4 steps (an even number of pairs does); the rest one step
    // per pass
    if (b->fuse && b->depth == 3) {
        const int triples = nsteps / 3;
        int rc = run_units(b, 4, triples);
        if (rc == LBM_OK) rc = run_units(b, npt_index(b->npt), nsteps - 3 * triples);
        return rc;
    }
    const int pairs = b->fuse ? 2 * (nsteps / 4) : 0;
    int rc = run_units(b, 3, pairs);
    if (rc == LBM_OK) rc = run_units(b, npt_index(b->npt), nsteps - 2 * pairs);
    return rc;
}

int lbm_batch_status(lbm_batch* b, long long* step, long long* blowup_steps) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    std::vector<int> flags((size_t)b->n);
    int err = 0;
    long long dstep = 0;
    int rc = check_hip(hipStreamSynchronize(b->stream), "synchronise");
    if (rc == LBM_OK) rc = check_hip(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost), "copy err");
    if (rc == LBM_OK) rc = check_hip(hipMemcpy(&dstep, b->d_step, sizeof(dstep), hipMemcpyDeviceToHost), "copy step");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(flags.data(), b->d_blowup, sizeof(int) * flags.size(), hipMemcpyDeviceToHost),
                       "copy blow-up steps");
    if (rc != LBM_OK) return rc;
    if (err == 2) return set_error(LBM_EHIP, "persistent launch stopped: an XCD that owns instances got no workgroup");
    if (err) return set_error(LBM_EHIP, "persistent launch stopped: a barrier timed out");
    if (dstep < b->step) return set_error(LBM_EHIP, "device step counter %lld behind %lld", dstep, b->step);
    b->step = dstep;  // ahead after replays of a captured run
    if (step) *step = b->step;
    if (blowup_steps)
        for (int j = 0; j < b->n; ++j) blowup_steps[j] = flags[j] == INT_MAX ? -1 : (long long)flags[j];
    return LBM_OK;
}

int lbm_batch_get_state(lbm_batch* b, int instance, double* f) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (instance < 0 || instance >= b->n) return set_error(LBM_EINVAL, "instance %d out of range", instance);
    if (!f) return set_error(LBM_EINVAL, "f is NULL");
    const lbm_instance_desc& d = b->hdesc[instance];
    const Launch l = launch_for(d.nx, d.ny);
    const Geom g{d.nx, d.ny, b->plane[instance]};
    // a live instance's state is in the copy of the step's parity; one that blew up or was
    // retired stopped advancing, and its state is in the copy its last pass wrote
    int blow = INT_MAX, ret = INT_MAX, last = 0;
    int rc = check_hip(hipStreamSynchronize(b->stream), "synchronise");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(&blow, b->d_blowup + instance, sizeof(int), hipMemcpyDeviceToHost), "copy blow-up");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(&ret, b->d_retired + instance, sizeof(int), hipMemcpyDeviceToHost), "copy retired");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(&last, b->d_lastcopy + instance, sizeof(int), hipMemcpyDeviceToHost), "copy last copy");
    long long dstep = 0;
    if (rc == LBM_OK) rc = check_hip(hipMemcpy(&dstep, b->d_step, sizeof(dstep), hipMemcpyDeviceToHost), "copy step");
    if (rc != LBM_OK) return rc;
    if (dstep > b->step) b->step = dstep;  // ahead after replays of a captured run
    const int sc = (blow == INT_MAX && ret == INT_MAX) ? (int)(b->step & 1) : last;
    const size_t eoff = (size_t)(sc * b->copy_elems + b->off[instance]);
    const Pop9 fref = reference_populations(storage_reference(b->prec, d.rho0, d.ux0, d.uy0), d.eq_order);
    switch (b->prec) {
        case LBM_F64:
            hipLaunchKernelGGL(k_batch_get<kF64>, l.grid, l.block, 0, b->stream,
                               reinterpret_cast<const double*>(b->buf) + eoff, g, fref, f);
            break;
        case LBM_F32_SHIFTED:
            hipLaunchKernelGGL(k_batch_get<kF32>, l.grid, l.block, 0, b->stream,
                               reinterpret_cast<const float*>(b->buf) + eoff, g, fref, f);
            break;
        default:
            hipLaunchKernelGGL(k_batch_get<kF16>, l.grid, l.block, 0, b->stream,
                               reinterpret_cast<const _Float16*>(b->buf) + eoff, g, fref, f);
            break;
    }
    return check_hip(hipGetLastError(), "batch get_state launch");
}

int lbm_batch_mean_u2(lbm_batch* b, double* mean_u2) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (!mean_u2) return set_error(LBM_EINVAL, "mean_u2 is NULL");
    const dim3 tiles(b->ntiles[0]), tb(kTileThreads), ib((b->n + 255) / 256), ibt(256);
    switch (b->prec) {
        case LBM_F64:
            hipLaunchKernelGGL(k_batch_u2_tiles<kF64>, tiles, tb, 0, b->stream,
                               reinterpret_cast<const double*>(b->buf), b->copy_elems, b->d_step,
                               reinterpret_cast<const BDesc<double>*>(b->d_desc[0]), b->d_tiles[0], b->d_u2part);
            hipLaunchKernelGGL(k_batch_u2_sum<double>, ib, ibt, 0, b->stream,
                               reinterpret_cast<const BDesc<double>*>(b->d_desc[0]), b->n, b->d_u2part, mean_u2);
            break;
        case LBM_F32_SHIFTED:
            hipLaunchKernelGGL(k_batch_u2_tiles<kF32>, tiles, tb, 0, b->stream,
                               reinterpret_cast<const float*>(b->buf), b->copy_elems, b->d_step,
                               reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->d_tiles[0], b->d_u2part);
            hipLaunchKernelGGL(k_batch_u2_sum<float>, ib, ibt, 0, b->stream,
                               reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->n, b->d_u2part, mean_u2);
            break;
        default:
            hipLaunchKernelGGL(k_batch_u2_tiles<kF16>, tiles, tb, 0, b->stream,
                               reinterpret_cast<const _Float16*>(b->buf), b->copy_elems, b->d_step,
                               reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->d_tiles[0], b->d_u2part);
            hipLaunchKernelGGL(k_batch_u2_sum<float>, ib, ibt, 0, b->stream,
                               reinterpret_cast<const BDesc<float>*>(b->d_desc[0]), b->n, b->d_u2part, mean_u2);
            break;
    }
    return check_hip(hipGetLastError(), "batch mean |u|^2 launch");
}

int lbm_batch_set_active(lbm_batch* b, const int* active) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (!active) return set_error(LBM_EINVAL, "active is NULL");
    hipLaunchKernelGGL(k_retire, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, active, b->d_active,
                       b->d_retired, b->n, b->d_step);
    return check_hip(hipGetLastError(), "batch set_active launch");
}

int lbm_batch_rebalance(lbm_batch* b) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    std::vector<char> live;
    const int rc = live_set(b, live);
    return rc != LBM_OK ? rc : deal_tables(b, live);
}

int lbm_batch_residency(lbm_batch* b, int shape, int* from_resources, int* occupancy_query, int* resident,
                        int* probe_stepdowns) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (shape < 0 || shape > 4) return set_error(LBM_EINVAL, "shape %d not in 0..4", shape);
    if (from_resources) *from_resources = b->res_fit[shape];
    if (occupancy_query) *occupancy_query = b->occ[shape];
    if (resident) *resident = b->resident[shape];
    if (probe_stepdowns) *probe_stepdowns = b->probe_stepdowns;
    return LBM_OK;
}

int lbm_batch_set_fusion(lbm_batch* b, int strip_rows) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (strip_rows < 0 || (strip_rows > 0 && (strip_rows % kBatchRing != 0 || strip_rows > (1 << 20))))
        return set_error(LBM_EINVAL, "strip_rows %d: 0 or a positive multiple of %d", strip_rows, kBatchRing);
    if (strip_rows == 0) {
        b->fuse = 0;
        return LBM_OK;
    }
    b->fuse = 1;
    if (strip_rows == b->hs) return LBM_OK;
    // live_set synchronises the stream first: no launch still reads the strip table when it is
    // reallocated and rewritten
    std::vector<char> live;
    int rc = live_set(b, live);
    if (rc != LBM_OK) return rc;
    b->hs = strip_rows;
    rc = alloc_strips(b);
    return rc != LBM_OK ? rc : deal_tables(b, live);
}

int lbm_batch_set_fusion_depth(lbm_batch* b, int steps) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (steps != 2 && steps != 3) return set_error(LBM_EINVAL, "steps per fused pass %d not in {2, 3}", steps);
    if (steps == 3 && !batch3_kernel_p(b->prec))
        return set_error(LBM_EUNSUPPORTED, "three steps per pass need an FP64 or FP32 batch");
    b->depth = steps;
    return LBM_OK;
}

int lbm_batch_get_fusion_depth(lbm_batch* b, int* steps) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (steps) *steps = b->depth;
    return LBM_OK;
}

int lbm_batch_get_fusion(lbm_batch* b, int* strip_rows) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (strip_rows) *strip_rows = b->fuse ? b->hs : 0;
    return LBM_OK;
}

int lbm_batch_set_launch(lbm_batch* b, int nodes_per_thread, int groups_per_cu) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (nodes_per_thread != 1 && nodes_per_thread != 2 && nodes_per_thread != 4)
        return set_error(LBM_EINVAL, "nodes_per_thread %d not in {1,2,4}", nodes_per_thread);
    if (groups_per_cu < 0) return set_error(LBM_EINVAL, "groups_per_cu %d < 0", groups_per_cu);
    b->npt = nodes_per_thread;
    b->gpc = groups_per_cu;
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, int trials, int* nodes_per_thread, int* groups_per_cu,
                       double* us_per_step) {
    if (!b) return set_error(LBM_ESTATE, "batch is NULL");
    if (trials < 1) return set_error(LBM_EINVAL, "trials %d < 1", trials);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (rc == LBM_OK) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
    const int npts[3] = {1, 2, 4};
    const int keep_npt = b->npt, keep_gpc = b->gpc, keep_fuse = b->fuse, keep_depth = b->depth;
    float best = 0.f;
    int best_npt = keep_npt, best_gpc = keep_gpc, best_fuse = keep_fuse, best_depth = keep_depth;
    // the timed passes run ahead of the step counter and may record a blow-up of a step not taken
    // yet: the records are restored afterwards
    std::vector<int> flags0((size_t)b->n);
    if (rc == LBM_OK) rc = check_hip(hipStreamSynchronize(b->stream), "synchronise");
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(flags0.data(), b->d_blowup, sizeof(int) * flags0.size(), hipMemcpyDeviceToHost),
                       "copy blow-up steps");
    // candidates: one step per pass (1, 2, 4 nodes per thread), then two and (FP64, FP32) three
    // steps per pass; each at the residency limit and at half of it; times per step
    const int nshapes = batch3_kernel_p(b->prec) ? 5 : 4;
    for (int k = 0; k < nshapes && rc == LBM_OK; ++k)
        for (int half = 0; half < 2 && rc == LBM_OK; ++half) {
            if (k < 3) b->npt = npts[k];
            rc = ensure_resident(b, k);
            if (rc != LBM_OK) break;
            const int lim = groups_limit(b, k);
            b->gpc = half ? std::max(1, lim / 2) : 0;
            if (half && b->gpc == lim) continue;
            rc = run_persistent(b, k, 1, 0);  // warm-up (non-advancing)
            if (rc == LBM_OK) rc = check_hip(hipEventRecord(e0, b->stream), "hipEventRecord");
            if (rc == LBM_OK) rc = run_persistent(b, k, trials, 0);
            if (rc == LBM_OK) rc = check_hip(hipEventRecord(e1, b->stream), "hipEventRecord");
            if (rc == LBM_OK) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            if (rc == LBM_OK) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (k == 3) ms *= 0.5f;
            if (k == 4) ms /= 3.f;
            int err = 0;
            if (rc == LBM_OK) rc = check_hip(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost), "copy err");
            if (rc == LBM_OK && err) rc = set_error(LBM_EHIP, "persistent launch stopped: a barrier timed out");
            if (rc == LBM_OK && (best == 0.f || ms < best)) {
                best = ms;
                best_npt = b->npt;
                best_gpc = b->gpc;
                best_fuse = k >= 3 ? 1 : 0;
                best_depth = k == 4 ? 3 : 2;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->npt = rc == LBM_OK ? best_npt : keep_npt;
    b->gpc = rc == LBM_OK ? best_gpc : keep_gpc;
    b->fuse = rc == LBM_OK ? best_fuse : keep_fuse;
    b->depth = rc == LBM_OK ? best_depth : keep_depth;
    if (rc == LBM_OK)
        rc = check_hip(hipMemcpy(b->d_blowup, flags0.data(), sizeof(int) * flags0.size(), hipMemcpyHostToDevice),
                       "restore blow-up steps");
    if (rc != LBM_OK) return rc;
    if (nodes_per_thread) *nodes_per_thread = best_npt;
    if (groups_per_cu) *groups_per_cu = best_gpc == 0 ? b->resident[shape_of(b, best_fuse)] : best_gpc;
    if (us_per_step) *us_per_step = 1e3 * (double)best / trials;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (int k = 0; k < 3; ++k) {
        if (b->d_desc[k]) (void)hipFree(b->d_desc[k]);
        if (b->d_tiles[k]) (void)hipFree(b->d_tiles[k]);
    }
    for (int k = 0; k < 5; ++k) {
        if (b->d_xtab[k]) (void)hipFree(b->d_xtab[k]);
        if (b->d_run[k]) (void)hipFree(b->d_run[k]);
    }
    if (b->d_lastcopy) (void)hipFree(b->d_lastcopy);
    if (b->d_blowup) (void)hipFree(b->d_blowup);
    if (b->d_active) (void)hipFree(b->d_active);
    if (b->d_retired) (void)hipFree(b->d_retired);
    if (b->d_u2part) (void)hipFree(b->d_u2part);
    if (b->d_bar) (void)hipFree(b->d_bar);
    if (b->d_err) (void)hipFree(b->d_err);
    if (b->d_step) (void)hipFree(b->d_step);
    delete b;
}

}  // extern "C"
