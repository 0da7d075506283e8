// Batched sweep: many independent periodic boxes (porous unit cells of uneven
// sizes, each with its own tau and force) advanced together by one persistent
// kernel that runs every step of a call, with a grid-wide barrier between
// steps.
//
// Layout: the items' cells are packed one after another, x fastest inside an
// item, and each population row spans all items: buf[i*Ntot + base_k + local]
// (Ntot: the packed cells plus the row pad, hlbm_config::row_pad_bytes of
// items[0]).
// The packed cells are cut into tiles of `tile` consecutive cells (one block
// of `tile` threads; the block size of every batched launch) that never
// straddle two items (a tile's tail past the item's end is masked).
//
// Work distribution of the persistent kernel: blocks take chunks of `chunk`
// consecutive tiles from one device-wide counter, in order, so the blocks
// resident at any moment work on one contiguous band of tiles (the rows a pull
// reads from the neighbouring y and z rows are still in L2 when the band
// reaches them) and a block that finishes early takes more (no static
// imbalance at the step's end).  Chunk k belongs to step k / nch (nch chunks
// per step); a block that draws a chunk of a later step keeps it and works on
// it in that step, after the grid barrier.  Each block draws its next chunk
// while it works on the current one.  (Drawing per block beat drawing per
// wavefront, whose four times as many draws contend on the counter.)  The
// grid is `blocks_per_cu` resident blocks per CU, at most what fits.  Every
// block takes part in every grid barrier, and each participant costs a cache
// write-back and invalidation, so fewer, busier blocks win: on the 256-cell
// workload 2 blocks of 256 threads per CU ran 10% faster than the 5 that fit.
// Tile size, blocks per CU and chunk are chosen by the autotuner; results do
// not depend on them.
// The barrier waits with a bounded spin; if the bound is exceeded (a block was
// never scheduled) or another block reported an error, every block leaves the
// kernel at its next barrier and the host sees the error flag, so the kernel
// always ends.
#include "cell.hpp"

namespace hlbm {

// Quotient of l by d via a 32-bit multiply-high, exact for l * d < 2^32
// (checked on the host for every item).
__device__ __forceinline__ uint32_t div_magic(uint32_t l, uint32_t magic) { return __umulhi(l, magic); }

__device__ __forceinline__ bool grid_barrier(unsigned long long* __restrict__ arrivals,
                                             unsigned long long target, int* __restrict__ err,
                                             unsigned spin_limit)
{
    __shared__ int ok;
    // Release.  Each wave waits until its own stores have completed (reached
    // L2: the vector L1 is write-through), the block barrier orders that
    // before thread 0, and thread 0 releases them at device scope -- one
    // write-back of this XCD's L2 per block, not per wave -- before it signals
    // arrival, so the step's results are visible to blocks on every XCD.
    // Release only: an acquire here would invalidate the L2 under blocks still
    // computing.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // the write-back must have completed before the arrival is counted
        __builtin_amdgcn_s_waitcnt(0);
        atomicAdd(arrivals, 1ull);
        int good = 1;
        unsigned spins = 0;
        // Relaxed polling (device-coherent loads, no cache invalidation per
        // poll); the acquire follows once, below.
        while (__hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                good = 0;
                break;
            }
            if (++spins > spin_limit) {
                atomicOr(err, 1);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        // acquire by the thread that observed the count ...
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    // ... and by every wave after the block barrier: drop stale copies of
    // other blocks' results from this CU's and this XCD's caches before the
    // next step reads them.
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

__global__ void batch_reset_kernel(unsigned long long* sync, int* err)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sync[0] = 0ull;
        sync[1] = 0ull;
        *err = 0;
    }
}

// One cell of one item: periodic pull inside the item's box, collision,
// store.  `l` is the cell's index inside the item.  MASKED: items may hold
// resolved solid cells (link mask over the packed cells; all zero for an item
// without obstacles, which then loads exactly what the periodic gather loads):
// bounce-back at solid links, zeros in solid cells.
template <class S, bool MASKED>
__device__ __forceinline__ void batch_cell(const typename S::T* __restrict__ src,
                                           typename S::T* __restrict__ dst,
                                           const typename S::D* __restrict__ dfield,
                                           const uint32_t* __restrict__ linkmask, uint32_t Ntot,
                                           const BatchItem& it, uint32_t l, typename S::R rho0,
                                           typename S::R scale, typename S::R inv_scale)
{
    using R = typename S::R;
    using L = D3Q19;
    const uint32_t t = div_magic(l, it.mx);
    const uint32_t x = l - t * it.nx;
    const uint32_t z = div_magic(t, it.my);
    const uint32_t y = t - z * it.ny;
    R g[L::Q];
    bool solid = false;
    if (MASKED)
        solid = gather_masked<L, S>(src, Ntot, linkmask, it.base, it.nx, it.ny, it.nz, x, y, z, inv_scale, g);
    else
        gather_periodic<L, S>(src, Ntot, it.base, it.nx, it.ny, it.nz, x, y, z, inv_scale, g);
    const uint32_t cell = it.base + l;
    const R d = S::load_d(ld(dfield, cell));
    R drho, ux, uy, uz;
    collide<L, R, ScalarShift<R>, S::exact_moments>(g, ScalarShift<R>{d}, R(it.F[0]), R(it.F[1]), R(it.F[2]), rho0, R(it.omega), R(it.pref), drho, ux,
                  uy, uz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        st_stream(dst + (size_t)i * Ntot, cell, S::store(MASKED ? sel(solid, R(0), g[i]) : g[i], scale));
}

template <class S, bool MASKED>
__global__ __launch_bounds__(TILE_MAX) void batch_persistent_kernel(
    typename S::T* __restrict__ buf_a, typename S::T* __restrict__ buf_b,
    const typename S::D* __restrict__ dfield, const uint32_t* __restrict__ linkmask,
    const BatchItem* __restrict__ items,
    const uint32_t* __restrict__ tile_item, uint32_t ntiles, uint32_t chunk, uint32_t Ntot, int nsteps,
    int start_in_b, double rho0_d, double scale_d, unsigned long long* __restrict__ sync,
    int* __restrict__ err, unsigned spin_limit)
{
    using R = typename S::R;
    const R rho0 = R(rho0_d), scale = R(scale_d), inv_scale = R(1.0 / scale_d);
    const uint32_t tile = blockDim.x;
    const unsigned long long nch = (ntiles + chunk - 1) / chunk;  // chunks per step
    __shared__ unsigned long long next;
    if (threadIdx.x == 0) next = atomicAdd(&sync[1], 1ull);
    __syncthreads();
    unsigned long long cur = next;
    for (int s = 0; s < nsteps; ++s) {
        const bool from_b = ((s + start_in_b) & 1) != 0;
        const typename S::T* __restrict__ src = from_b ? buf_b : buf_a;
        typename S::T* __restrict__ dst = from_b ? buf_a : buf_b;
        const unsigned long long first = (unsigned long long)s * nch;
        while (cur < first + nch) {
            // draw the following chunk now; its number is needed only after
            // this chunk is done
            unsigned long long drawn = 0ull;
            if (threadIdx.x == 0) drawn = atomicAdd(&sync[1], 1ull);
            const uint32_t t0 = (uint32_t)(cur - first) * chunk;
            const uint32_t t1 = min(ntiles, t0 + chunk);
            for (uint32_t t = t0; t < t1; ++t) {
                const BatchItem it = items[tile_item[t]];
                const uint32_t l = (t - it.tile0) * tile + threadIdx.x;
                if (l < it.cells)
                    batch_cell<S, MASKED>(src, dst, dfield, linkmask, Ntot, it, l, rho0, scale, inv_scale);
            }
            __syncthreads();  // every thread has read `next` for this chunk
            if (threadIdx.x == 0) next = drawn;
            __syncthreads();
            cur = next;
        }
        if (s + 1 < nsteps &&
            !grid_barrier(&sync[0], (unsigned long long)(s + 1) * gridDim.x, err, spin_limit))
            return;
    }
}

// One launch per step over all tiles (no barrier); used for the non-persistent
// form and as the reference the persistent form must match bit for bit.
template <class S, bool MASKED>
__global__ __launch_bounds__(TILE_MAX) void batch_step_kernel(
    const typename S::T* __restrict__ src, typename S::T* __restrict__ dst,
    const typename S::D* __restrict__ dfield, const uint32_t* __restrict__ linkmask,
    const BatchItem* __restrict__ items, const uint32_t* __restrict__ tile_item, uint32_t Ntot,
    double rho0_d, double scale_d)
{
    using R = typename S::R;
    const uint32_t t = blockIdx.x;
    const BatchItem it = items[tile_item[t]];
    const uint32_t l = (t - it.tile0) * blockDim.x + threadIdx.x;
    if (l < it.cells)
        batch_cell<S, MASKED>(src, dst, dfield, linkmask, Ntot, it, l, R(rho0_d), R(scale_d), R(1.0 / scale_d));
}

// Moments of every item at the current time level: one block per tile writes
// FP64 partials (sum drho, sum rho u); optionally the fields of one item.
template <class S, bool MASKED>
__global__ __launch_bounds__(TILE_MAX) void batch_moments_kernel(
    const typename S::T* __restrict__ src, const uint32_t* __restrict__ linkmask,
    const BatchItem* __restrict__ items, const uint32_t* __restrict__ tile_item, uint32_t Ntot,
    double rho0_d, double scale_d, double* __restrict__ partials, int sel_item,
    double* __restrict__ drho_out, double* __restrict__ u_out)
{
    using R = typename S::R;
    using L = D3Q19;
    const uint32_t t = blockIdx.x;
    const uint32_t k = tile_item[t];
    const BatchItem it = items[k];
    const uint32_t l = (t - it.tile0) * blockDim.x + threadIdx.x;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (l < it.cells) {
        const uint32_t q = div_magic(l, it.mx);
        const uint32_t x = l - q * it.nx;
        const uint32_t z = div_magic(q, it.my);
        const uint32_t y = q - z * it.ny;
        R g[L::Q];
        bool solid = false;
        if (MASKED)
            solid = gather_masked<L, S>(src, Ntot, linkmask, it.base, it.nx, it.ny, it.nz, x, y, z,
                                        R(1.0 / scale_d), g);
        else
            gather_periodic<L, S>(src, Ntot, it.base, it.nx, it.ny, it.nz, x, y, z, R(1.0 / scale_d), g);
        R drho, ux, uy, uz;
        moments_of<L, R, S::exact_moments>(g, R(it.F[0]), R(it.F[1]), R(it.F[2]), R(rho0_d), drho, ux, uy, uz);
        // solid cells report zeros and add nothing to the totals
        drho = sel(solid, R(0), drho);
        ux = sel(solid, R(0), ux);
        uy = sel(solid, R(0), uy);
        uz = sel(solid, R(0), uz);
        const double rho = rho0_d + (double)drho;
        m0 = (double)drho;
        m1 = rho * (double)ux;
        m2 = rho * (double)uy;
        m3 = rho * (double)uz;
        if ((int)k == sel_item && drho_out) {
            drho_out[l] = (double)drho;
            u_out[l] = (double)ux;
            u_out[(size_t)it.cells + l] = (double)uy;
            u_out[2 * (size_t)it.cells + l] = (double)uz;
        }
    }
    block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)t);
}

// Per-item totals: block k sums the partials of item k's tiles in order.
__global__ __launch_bounds__(256) void batch_item_reduce_kernel(const double* __restrict__ partials,
                                                                const BatchItem* __restrict__ items,
                                                                uint32_t tile, double* __restrict__ totals)
{
    const BatchItem it = items[blockIdx.x];
    const uint32_t nt = (it.cells + tile - 1) / tile;
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (uint32_t j = threadIdx.x; j < nt; j += blockDim.x) {
        const double* p = partials + 4 * (size_t)(it.tile0 + j);
        a += p[0];
        b += p[1];
        c += p[2];
        d += p[3];
    }
    block_sum4(a, b, c, d, totals + 4 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Calls f.template operator()<S, MASKED>() for the storage code and whether a
// link mask is present.
template <class F>
static hipError_t with_storage(int storage, bool masked, F&& f)
{
    switch (storage) {
    case StoreF32::code: return masked ? f.template run<StoreF32, true>() : f.template run<StoreF32, false>();
    case StoreF16S::code: return masked ? f.template run<StoreF16S, true>() : f.template run<StoreF16S, false>();
    case StoreBF16S::code:
        return masked ? f.template run<StoreBF16S, true>() : f.template run<StoreBF16S, false>();
    case StoreF64::code: return masked ? f.template run<StoreF64, true>() : f.template run<StoreF64, false>();
    default: return hipErrorInvalidValue;
    }
}

struct PersistentLaunch {
    const BatchLaunch& b;
    void *buf_a, *buf_b;
    const void* dfield;
    int nsteps, start_in_b;
    hipStream_t s;
    template <class S, bool M>
    hipError_t run() const
    {
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b.sync, b.err);
        hipLaunchKernelGGL((batch_persistent_kernel<S, M>), dim3(b.grid), dim3(b.tile), 0, s,
                           static_cast<typename S::T*>(buf_a), static_cast<typename S::T*>(buf_b),
                           static_cast<const typename S::D*>(dfield), b.linkmask, b.items, b.tile_item,
                           b.ntiles, b.chunk, b.Ntot, nsteps, start_in_b, b.rho0, b.scale, b.sync, b.err,
                           b.spin_limit);
        return hipGetLastError();
    }
};

hipError_t launch_batch_persistent(int storage, const BatchLaunch& b, void* buf_a, void* buf_b,
                                   const void* dfield, int nsteps, int start_in_b, hipStream_t s)
{
    return with_storage(storage, b.linkmask != nullptr,
                        PersistentLaunch{b, buf_a, buf_b, dfield, nsteps, start_in_b, s});
}

struct StepLaunch {
    const BatchLaunch& b;
    const void* src;
    void* dst;
    const void* dfield;
    hipStream_t s;
    template <class S, bool M>
    hipError_t run() const
    {
        hipLaunchKernelGGL((batch_step_kernel<S, M>), dim3(b.ntiles), dim3(b.tile), 0, s,
                           static_cast<const typename S::T*>(src), static_cast<typename S::T*>(dst),
                           static_cast<const typename S::D*>(dfield), b.linkmask, b.items, b.tile_item, b.Ntot,
                           b.rho0, b.scale);
        return hipGetLastError();
    }
};

hipError_t launch_batch_step(int storage, const BatchLaunch& b, const void* src, void* dst,
                             const void* dfield, hipStream_t s)
{
    return with_storage(storage, b.linkmask != nullptr, StepLaunch{b, src, dst, dfield, s});
}

struct MomentsLaunch {
    const BatchLaunch& b;
    const void* src;
    double* partials;
    int sel_item;
    double *drho, *u, *totals;
    hipStream_t s;
    template <class S, bool M>
    hipError_t run() const
    {
        hipLaunchKernelGGL((batch_moments_kernel<S, M>), dim3(b.ntiles), dim3(b.tile), 0, s,
                           static_cast<const typename S::T*>(src), b.linkmask, b.items, b.tile_item, b.Ntot,
                           b.rho0, b.scale, partials, sel_item, drho, u);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(batch_item_reduce_kernel, dim3(b.n_items), dim3(256), 0, s, partials, b.items,
                           b.tile, totals);
        return hipGetLastError();
    }
};

hipError_t launch_batch_moments(int storage, const BatchLaunch& b, const void* src, double* partials,
                                int sel_item, double* drho, double* u, double* totals, hipStream_t s)
{
    return with_storage(storage, b.linkmask != nullptr, MomentsLaunch{b, src, partials, sel_item, drho, u, totals, s});
}

// Executable graphs, built from explicit kernel nodes so that they can be
// launched on any stream, the legacy default stream included.  No memset
// nodes: the barrier reset is a kernel.
//   steps:      one node of the per-step kernel per step, each depending on
//               the one before (buffers alternate from node to node);
//   persistent: a reset node, then the persistent kernel for all steps.
struct GraphBuild {
    const BatchLaunch& b;
    void *buf_a, *buf_b;
    const void* dfield;
    int nsteps, start_in_b;
    bool persistent;
    hipGraphExec_t* out;
    template <class S, bool M>
    hipError_t run() const
    {
        hipGraph_t g = nullptr;
        hipError_t e = hipGraphCreate(&g, 0);
        if (e != hipSuccess) return e;
        auto* pa = static_cast<typename S::T*>(buf_a);
        auto* pb = static_cast<typename S::T*>(buf_b);
        auto* pd = static_cast<const typename S::D*>(dfield);
        const uint32_t* lm = b.linkmask;
        const BatchItem* items = b.items;
        const uint32_t* tile_item = b.tile_item;
        uint32_t ntiles = b.ntiles, chunk = b.chunk, Ntot = b.Ntot;
        double rho0 = b.rho0, scale = b.scale;
        unsigned long long* sync = b.sync;
        int* err = b.err;
        unsigned spin = b.spin_limit;
        int steps = nsteps, start = start_in_b;
        if (persistent) {
            void* reset_args[] = {&sync, &err};
            hipKernelNodeParams rp = {};
            rp.func = reinterpret_cast<void*>(batch_reset_kernel);
            rp.gridDim = dim3(1);
            rp.blockDim = dim3(64);
            rp.kernelParams = reset_args;
            hipGraphNode_t n_reset = nullptr, n_run = nullptr;
            e = hipGraphAddKernelNode(&n_reset, g, nullptr, 0, &rp);
            void* run_args[] = {&pa, &pb, &pd, &lm, &items, &tile_item, &ntiles, &chunk, &Ntot, &steps,
                                &start, &rho0, &scale, &sync, &err, &spin};
            hipKernelNodeParams kp = {};
            kp.func = reinterpret_cast<void*>(batch_persistent_kernel<S, M>);
            kp.gridDim = dim3(b.grid);
            kp.blockDim = dim3(b.tile);
            kp.kernelParams = run_args;
            if (e == hipSuccess) e = hipGraphAddKernelNode(&n_run, g, &n_reset, 1, &kp);
        } else {
            // node k reads the buffer written by node k - 1; the arguments are
            // copied when the node is added
            hipGraphNode_t prev = nullptr;
            for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
                const bool from_b = ((k + start_in_b) & 1) != 0;
                const typename S::T* src = from_b ? pb : pa;
                typename S::T* dst = from_b ? pa : pb;
                void* args[] = {&src, &dst, &pd, &lm, &items, &tile_item, &Ntot, &rho0, &scale};
                hipKernelNodeParams kp = {};
                kp.func = reinterpret_cast<void*>(batch_step_kernel<S, M>);
                kp.gridDim = dim3(b.ntiles);
                kp.blockDim = dim3(b.tile);
                kp.kernelParams = args;
                hipGraphNode_t node = nullptr;
                e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
                prev = node;
            }
        }
        if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        return e;
    }
};

hipError_t build_batch_graph(int storage, const BatchLaunch& b, void* buf_a, void* buf_b,
                             const void* dfield, int nsteps, int start_in_b, bool persistent, hipGraphExec_t* out)
{
    return with_storage(storage, b.linkmask != nullptr,
                        GraphBuild{b, buf_a, buf_b, dfield, nsteps, start_in_b, persistent, out});
}

struct Occupancy {
    int tile;
    int* blocks_per_cu;
    template <class S, bool M>
    hipError_t run() const
    {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_persistent_kernel<S, M>, tile, 0);
    }
};

// Resident blocks of `tile` threads per CU of the persistent kernel: the
// fewer of the unmasked and the masked form, so that a schedule stays valid
// when obstacles are added.
hipError_t batch_occupancy(int storage, int tile, int* blocks_per_cu)
{
    int plain = 0, masked = 0;
    hipError_t e = with_storage(storage, false, Occupancy{tile, &plain});
    if (e == hipSuccess) e = with_storage(storage, true, Occupancy{tile, &masked});
    *blocks_per_cu = plain < masked ? plain : masked;
    return e;
}

}  // namespace hlbm
