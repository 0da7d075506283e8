// Fused pull-stream + collide sweep of the homogenized lattice BGK scheme,
// moments gather, FP64 reductions and porosity conversion, for gfx950.
//
// Memory layout: structure of arrays, population i of cell c at
// buf[i*N + c], c = x + nx*(y + ny*z).  One thread owns one cell; a block
// covers `bx` consecutive cells of one x-row, so every population row is read
// by exactly one block and each load instruction of a wavefront is a
// contiguous (possibly one-element shifted) 64-lane run.  The sweep reads each
// post-collision population once (from x - c_i) and writes each new one once:
// 2*Q elements plus one porosity value per cell, the algorithmic minimum.
// Row offsets depend only on (y, z), which are uniform per block, so they are
// scalar; per-population bases are 64-bit uniform pointers and the per-lane
// offset is a 32-bit cell index.
#include "cell.hpp"

namespace hlbm {

// ---------------------------------------------------------------------------
// The sweep.  One step: pull, moments, shift, equilibrium, relax + force,
// store into the other buffer.  Returns the pre-collision moments (time level
// of `src`) and whether the cell is solid.
// ---------------------------------------------------------------------------
template <class L, class S, int BC>
__device__ __forceinline__ bool sweep_cell(const typename S::T* __restrict__ src,
                                           typename S::T* __restrict__ dst,
                                           const typename S::D* __restrict__ dfield, const Params& p,
                                           uint32_t x, uint32_t y, uint32_t z, typename S::R& drho,
                                           typename S::R& ux, typename S::R& uy, typename S::R& uz)
{
    using R = typename S::R;
    const uint32_t N = p.N;
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const R inv_scale = R(p.inv_scale), scale = R(p.scale);
    const R F0 = R(p.F[0]), F1 = R(p.F[1]), F2 = R(p.F[2]);
    const R rho0 = R(p.rho0), omega = R(p.omega), pref = R(p.pref);
    R g[L::Q];
    if (BC == BC_PERIODIC) {
        gather_periodic<L, S>(src, N, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
    } else {
        const Box b = box_of(p);
        const OpenFaces<R> of{rho0, R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                              R(p.outlet_rho)};
        gather_general<L, S>(src, N, b, of, (int)x, (int)y, (int)z, inv_scale, g);
    }
    const R d = S::load_d(ld(dfield, cell));
    collide<L, R>(g, d, F0, F1, F2, rho0, omega, pref, drho, ux, uy, uz);
    // solid cells (wall layers) hold zeros; selected, not branched
    bool solid = false;
    if (BC != BC_PERIODIC) solid = in_wall_layer(box_of(p), (int)x, (int)y, (int)z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) st(dst + (size_t)i * N, cell, S::store(sel(solid, R(0), g[i]), scale));
    return solid;
}

template <class L, class S, int BC>
__global__ __launch_bounds__(1024) void sweep_kernel(const typename S::T* __restrict__ src,
                                                      typename S::T* __restrict__ dst,
                                                      const typename S::D* __restrict__ dfield,
                                                      Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    R drho, ux, uy, uz;
    (void)sweep_cell<L, S, BC>(src, dst, dfield, p, x, blockIdx.y, blockIdx.z, drho, ux, uy, uz);
}

// The same step on a diagnostic step: the sweep also reduces the moments it
// has formed (time level of `src`, fluid cells) to FP64 block partials
// [sum drho, sum rho u_x, sum rho u_y, sum rho u_z], with the same block
// geometry and arithmetic as the moments kernel's totals.
template <class L, class S, int BC>
__global__ __launch_bounds__(1024) void sweep_diag_kernel(const typename S::T* __restrict__ src,
                                                           typename S::T* __restrict__ dst,
                                                           const typename S::D* __restrict__ dfield,
                                                           double* __restrict__ partials, Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (x < (uint32_t)p.nx) {
        R drho, ux, uy, uz;
        const bool solid =
            sweep_cell<L, S, BC>(src, dst, dfield, p, x, blockIdx.y, blockIdx.z, drho, ux, uy, uz);
        const double rho = p.rho0 + (double)drho;
        m0 = sel(solid, 0.0, (double)drho);
        m1 = sel(solid, 0.0, rho * (double)ux);
        m2 = sel(solid, 0.0, rho * (double)uy);
        m3 = sel(solid, 0.0, rho * (double)uz);
    }
    const uint32_t bk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)bk);
}

// Moments at the current time level (gather + moments, no collision).
template <class L, class S, int BC, class O>
__global__ __launch_bounds__(1024) void moments_kernel(const typename S::T* __restrict__ src,
                                                        O* __restrict__ drho_out,
                                                        O* __restrict__ u_out,
                                                        double* __restrict__ partials, Params p)
{
    using R = typename S::R;
    const uint32_t N = p.N;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const R inv_scale = R(p.inv_scale);
    const R F0 = R(p.F[0]), F1 = R(p.F[1]), F2 = R(p.F[2]), rho0 = R(p.rho0);
    const double rho0d = p.rho0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (x < (uint32_t)p.nx) {
        const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
        R g[L::Q];
        bool fluid = true;
        if (BC == BC_PERIODIC) {
            gather_periodic<L, S>(src, N, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
        } else {
            const Box b = box_of(p);
            fluid = !in_wall_layer(b, (int)x, (int)y, (int)z);
            const OpenFaces<R> of{rho0, R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                                  R(p.outlet_rho)};
            gather_general<L, S>(src, N, b, of, (int)x, (int)y, (int)z, inv_scale, g);
        }
        R drho, ux, uy, uz;
        moments_of<L, R>(g, F0, F1, F2, rho0, drho, ux, uy, uz);
        drho = sel(fluid, drho, R(0));
        ux = sel(fluid, ux, R(0));
        uy = sel(fluid, uy, R(0));
        uz = sel(fluid, uz, R(0));
        if (drho_out) drho_out[cell] = O(drho);
        if (u_out) {
            u_out[cell] = O(ux);
            u_out[(size_t)N + cell] = O(uy);
            u_out[2 * (size_t)N + cell] = O(uz);
        }
        const double rho = rho0d + (double)drho;
        m0 = (double)drho;
        m1 = sel(fluid, rho * (double)ux, 0.0);
        m2 = sel(fluid, rho * (double)uy, 0.0);
        m3 = sel(fluid, rho * (double)uz, 0.0);
    }
    if (partials) {
        const uint32_t bk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)bk);
    }
}

// Reduction of per-block partials in a fixed order (deterministic), in two
// passes: block b of the first pass sums the contiguous chunk
// [b*chunk, (b+1)*chunk) of the partials; one block then sums those results.
__global__ __launch_bounds__(256) void reduce4_kernel(const double* __restrict__ partials,
                                                      uint32_t n, uint32_t chunk,
                                                      double* __restrict__ out)
{
    const uint32_t begin = blockIdx.x * chunk;
    const uint32_t end = min(n, begin + chunk);
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (uint32_t k = begin + threadIdx.x; k < end; k += blockDim.x) {
        a += partials[4 * (size_t)k + 0];
        b += partials[4 * (size_t)k + 1];
        c += partials[4 * (size_t)k + 2];
        d += partials[4 * (size_t)k + 3];
    }
    block_sum4(a, b, c, d, out + 4 * (size_t)blockIdx.x);
}

// Porosity conversion with validation: d must be finite and in [0, 1].  A
// block holding an invalid value sets *flag (cleared by the caller).
template <class I, class O>
__global__ __launch_bounds__(256) void porosity_kernel(const I* __restrict__ in, O* __restrict__ out,
                                                       uint32_t n, int* __restrict__ flag)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (k < n) {
        const double v = (double)in[k];
        bad = !(v >= 0.0 && v <= 1.0);  // also catches NaN
        out[k] = O(in[k]);
    }
    const int any = __syncthreads_or(bad);
    if (threadIdx.x == 0 && any) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
Launch cell_launch(const Params& p, int bx)
{
    Launch l;
    l.block = dim3(bx, 1, 1);
    l.grid = dim3((p.nx + bx - 1) / bx, p.ny, p.nz);
    l.nblocks = l.grid.x * l.grid.y * l.grid.z;
    return l;
}

template <class L, class S>
static hipError_t sweep_dispatch_bc(int bcmode, const Params& p, const void* src, void* dst,
                                    const void* dfield, int bx, hipStream_t s, double* diag)
{
    const Launch l = cell_launch(p, bx);
    auto* a = static_cast<const typename S::T*>(src);
    auto* b = static_cast<typename S::T*>(dst);
    auto* d = static_cast<const typename S::D*>(dfield);
    if (diag) {
        if (bcmode == BC_PERIODIC)
            hipLaunchKernelGGL((sweep_diag_kernel<L, S, BC_PERIODIC>), l.grid, l.block, 0, s, a, b, d, diag, p);
        else
            hipLaunchKernelGGL((sweep_diag_kernel<L, S, BC_GENERAL>), l.grid, l.block, 0, s, a, b, d, diag, p);
    } else if (bcmode == BC_PERIODIC) {
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_PERIODIC>), l.grid, l.block, 0, s, a, b, d, p);
    } else {
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_GENERAL>), l.grid, l.block, 0, s, a, b, d, p);
    }
    return hipGetLastError();
}

template <class L>
static hipError_t sweep_dispatch_store(int storage, int bcmode, const Params& p, const void* src,
                                       void* dst, const void* dfield, int bx, hipStream_t s,
                                       double* diag)
{
    switch (storage) {
    case StoreF64::code: return sweep_dispatch_bc<L, StoreF64>(bcmode, p, src, dst, dfield, bx, s, diag);
    case StoreF32::code: return sweep_dispatch_bc<L, StoreF32>(bcmode, p, src, dst, dfield, bx, s, diag);
    case StoreF16S::code: return sweep_dispatch_bc<L, StoreF16S>(bcmode, p, src, dst, dfield, bx, s, diag);
    case StoreBF16S::code: return sweep_dispatch_bc<L, StoreBF16S>(bcmode, p, src, dst, dfield, bx, s, diag);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int q, int storage, int bcmode, const Params& p, const void* src, void* dst,
                        const void* dfield, int bx, hipStream_t s, double* diag_partials)
{
    if (q == 9) return sweep_dispatch_store<D2Q9>(storage, bcmode, p, src, dst, dfield, bx, s, diag_partials);
    if (q == 19) return sweep_dispatch_store<D3Q19>(storage, bcmode, p, src, dst, dfield, bx, s, diag_partials);
    return hipErrorInvalidValue;
}

template <class L, class S, class O>
static hipError_t moments_dispatch_bc(int bcmode, const Params& p, const void* src, void* drho,
                                      void* u, double* partials, int bx, hipStream_t s)
{
    const Launch l = cell_launch(p, bx);
    auto* a = static_cast<const typename S::T*>(src);
    if (bcmode == BC_PERIODIC)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_PERIODIC, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    else
        hipLaunchKernelGGL((moments_kernel<L, S, BC_GENERAL, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    return hipGetLastError();
}

template <class L, class S>
static hipError_t moments_dispatch_out(int out_f64, int bcmode, const Params& p, const void* src,
                                       void* drho, void* u, double* partials, int bx,
                                       hipStream_t s)
{
    if (out_f64) return moments_dispatch_bc<L, S, double>(bcmode, p, src, drho, u, partials, bx, s);
    return moments_dispatch_bc<L, S, float>(bcmode, p, src, drho, u, partials, bx, s);
}

template <class L>
static hipError_t moments_dispatch_store(int storage, int out_f64, int bcmode, const Params& p,
                                         const void* src, void* drho, void* u, double* partials,
                                         int bx, hipStream_t s)
{
    switch (storage) {
    case StoreF64::code:
        return moments_dispatch_out<L, StoreF64>(out_f64, bcmode, p, src, drho, u, partials, bx, s);
    case StoreF32::code:
        return moments_dispatch_out<L, StoreF32>(out_f64, bcmode, p, src, drho, u, partials, bx, s);
    case StoreF16S::code:
        return moments_dispatch_out<L, StoreF16S>(out_f64, bcmode, p, src, drho, u, partials, bx, s);
    case StoreBF16S::code:
        return moments_dispatch_out<L, StoreBF16S>(out_f64, bcmode, p, src, drho, u, partials, bx, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moments(int q, int storage, int bcmode, const Params& p, const void* src,
                          void* drho, void* u, int out_f64, double* partials, int bx, hipStream_t s)
{
    if (q == 9)
        return moments_dispatch_store<D2Q9>(storage, out_f64, bcmode, p, src, drho, u, partials, bx, s);
    if (q == 19)
        return moments_dispatch_store<D3Q19>(storage, out_f64, bcmode, p, src, drho, u, partials, bx, s);
    return hipErrorInvalidValue;
}

hipError_t launch_reduce4(const double* partials, uint32_t nblocks, double* stage, double* out,
                          hipStream_t s)
{
    // first pass: at most REDUCE_STAGE blocks of >= 1024 partials each
    uint32_t g = (nblocks + 1023) / 1024;
    if (g > REDUCE_STAGE) g = REDUCE_STAGE;
    if (g <= 1) {
        hipLaunchKernelGGL(reduce4_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, nblocks, out);
        return hipGetLastError();
    }
    const uint32_t chunk = (nblocks + g - 1) / g;
    hipLaunchKernelGGL(reduce4_kernel, dim3(g), dim3(256), 0, s, partials, nblocks, chunk, stage);
    hipLaunchKernelGGL(reduce4_kernel, dim3(1), dim3(256), 0, s, (const double*)stage, g, g, out);
    return hipGetLastError();
}

template <class I>
static hipError_t porosity_dispatch_out(const void* in, int storage, void* out, uint32_t n, int* flag,
                                        hipStream_t s)
{
    const uint32_t nb = (n + 255) / 256;
    auto* src = static_cast<const I*>(in);
    if (storage == StoreF64::code)
        hipLaunchKernelGGL((porosity_kernel<I, double>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<double*>(out), n, flag);
    else if (storage == StoreF32::code)
        hipLaunchKernelGGL((porosity_kernel<I, float>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<float*>(out), n, flag);
    else
        hipLaunchKernelGGL((porosity_kernel<I, _Float16>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<_Float16*>(out), n, flag);
    return hipGetLastError();
}

hipError_t launch_porosity_convert(int in_dtype, const void* in, int storage, void* out, uint32_t n,
                                   int* flag, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    if (in_dtype == 0) return porosity_dispatch_out<double>(in, storage, out, n, flag, s);
    if (in_dtype == 1) return porosity_dispatch_out<float>(in, storage, out, n, flag, s);
    return porosity_dispatch_out<_Float16>(in, storage, out, n, flag, s);
}

}  // namespace hlbm
