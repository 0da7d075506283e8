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
#include "hlbm_internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

namespace hlbm {

// Element `idx` of a population row addressed by a 32-bit byte offset from a
// uniform base.  The host guarantees N * sizeof(T) < 2^32, so the offset cannot
// wrap; this lets every access use the scalar-base + 32-bit vector-offset
// form of global loads and stores.
template <class T>
__device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}

template <class T>
__device__ __forceinline__ void st(T* __restrict__ base, uint32_t idx, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)) = v;
}

// ---------------------------------------------------------------------------
// Collision of one fluid cell in the arithmetic type R (Sec. 3.2: BGK toward
// the homogenized Maxwellian; the velocity argument is (1 - d) u).
//   rho = rho0 + sum g, j = sum c g, u = (j + F/2)/rho, u_eq = (1 - d) u
//   g_i <- g_i - omega (g_i - g^eq_i(rho, u_eq)) + S_i
//   g^eq_i = w_i [ drho + rho (3 c.u_eq + 9/2 (c.u_eq)^2 - 3/2 u_eq.u_eq) ]
//   S_i    = (1 - 1/(2 tau)) w_i [ 3 (c_i - u).F + 9 (c_i.u)(c_i.F) ]
// Returns drho and u (the reported moments) through the reference arguments.
// ---------------------------------------------------------------------------
template <class L, class R>
__device__ __forceinline__ void collide(R (&g)[L::Q], R d, R F0, R F1, R F2, R rho0, R omega,
                                        R pref, R& drho_out, R& ux_out, R& uy_out, R& uz_out)
{
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        drho += g[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? g[i] : -g[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? g[i] : -g[i];
        if (L::cz[i]) jz += L::cz[i] > 0 ? g[i] : -g[i];
    }
    const R rho = rho0 + drho;
    const R inv_rho = R(1) / rho;
    const R ux = (jx + R(0.5) * F0) * inv_rho;
    const R uy = (jy + R(0.5) * F1) * inv_rho;
    const R uz = (jz + R(0.5) * F2) * inv_rho;
    const R sh = R(1) - d;
    const R ex = sh * ux, ey = sh * uy, ez = sh * uz;
    const R uu = ex * ex + ey * ey + ez * ez;
    const R uF = ux * F0 + uy * F1 + uz * F2;
    const R base = drho - R(1.5) * rho * uu;  // common part of every g^eq_i / w_i
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const R cx = R(L::cx[i]), cy = R(L::cy[i]), cz = R(L::cz[i]);
        const R w = R(L::w[i]);
        const R ce = cx * ex + cy * ey + cz * ez;
        const R cu = cx * ux + cy * uy + cz * uz;
        const R cF = cx * F0 + cy * F1 + cz * F2;
        const R geq = w * (base + rho * (R(3) * ce + R(4.5) * ce * ce));
        const R S = pref * w * (R(3) * (cF - uF) + R(9) * cu * cF);
        g[i] = g[i] - omega * (g[i] - geq) + S;
    }
    drho_out = drho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
}

// Moments only (no collision), same definitions as in collide().
template <class L, class R>
__device__ __forceinline__ void moments_of(const R (&g)[L::Q], R F0, R F1, R F2, R rho0, R& drho,
                                           R& ux, R& uy, R& uz)
{
    R s = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        s += g[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? g[i] : -g[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? g[i] : -g[i];
        if (L::cz[i]) jz += L::cz[i] > 0 ? g[i] : -g[i];
    }
    const R rho = rho0 + s;
    const R inv_rho = R(1) / rho;
    drho = s;
    ux = (jx + R(0.5) * F0) * inv_rho;
    uy = (jy + R(0.5) * F1) * inv_rho;
    uz = (jz + R(0.5) * F2) * inv_rho;
}

// ---------------------------------------------------------------------------
// Pull gather, fully periodic box: g*_i(x) = g_i(x - c_i) with wrap.
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ void gather_periodic(const typename S::T* __restrict__ src,
                                                const Params& p, uint32_t x, uint32_t y,
                                                uint32_t z, typename S::R inv_scale,
                                                typename S::R (&g)[L::Q])
{
    const uint32_t nx = p.nx, ny = p.ny, nz = p.nz;
    // Source coordinate for c = -1, 0, +1 (index c + 1): x - c with wrap.
    const uint32_t xs[3] = {x + 1 == nx ? 0u : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const typename S::T* __restrict__ pi = src + (size_t)i * p.N;
        const uint32_t off = xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        g[i] = S::load(ld(pi, off), inv_scale);
    }
}

// Source cell in a wall layer?  (A wall face makes its first/last layer solid.)
__device__ __forceinline__ bool in_wall_layer(const Params& p, int sx, int sy, int sz)
{
    return (p.bc_lo[0] == 1 && sx == 0) || (p.bc_hi[0] == 1 && sx == p.nx - 1) ||
           (p.bc_lo[1] == 1 && sy == 0) || (p.bc_hi[1] == 1 && sy == p.ny - 1) ||
           (p.bc_lo[2] == 1 && sz == 0) || (p.bc_hi[2] == 1 && sz == p.nz - 1);
}

// Shifted second-order equilibrium of one population (open faces only).
template <class L, class R>
__device__ __forceinline__ R feq_shifted(int i, R rho, R rho0, R ux, R uy, R uz)
{
    const R cu = R(L::cx[i]) * ux + R(L::cy[i]) * uy + R(L::cz[i]) * uz;
    const R uu = ux * ux + uy * uy + uz * uz;
    return R(L::w[i]) * ((rho - rho0) + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
}

// ---------------------------------------------------------------------------
// Pull gather with walls and open faces.  Returns false for a solid cell.
//   * periodic axes wrap;
//   * a source in a wall layer -> halfway bounce-back g*_i(x) = g_opp(i)(x)
//     (takes precedence on edges);
//   * a source beyond an open face (lowest axis first) -> equilibrium from the
//     cell's own post-collision state: inlet f^eq(rho_b, u_in), outlet
//     f^eq(rho_out, j_b/rho_b), shifted by w rho0.
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ bool gather_general(const typename S::T* __restrict__ src,
                                               const Params& p, int x, int y, int z,
                                               typename S::R inv_scale,
                                               typename S::R (&g)[L::Q])
{
    using R = typename S::R;
    if (in_wall_layer(p, x, y, z)) return false;
    const uint32_t cell = (uint32_t)x + (uint32_t)p.nx * ((uint32_t)y + (uint32_t)p.ny * (uint32_t)z);
    const int n[3] = {p.nx, p.ny, p.nz};
    const int X[3] = {x, y, z};
    const bool on_open = (p.bc_lo[0] >= 2 && x == 0) || (p.bc_hi[0] >= 2 && x == p.nx - 1) ||
                         (p.bc_lo[1] >= 2 && y == 0) || (p.bc_hi[1] >= 2 && y == p.ny - 1) ||
                         (p.bc_lo[2] >= 2 && z == 0) || (p.bc_hi[2] >= 2 && z == p.nz - 1);
    R rho_b = R(p.rho0), jbx = R(0), jby = R(0), jbz = R(0);
    if (on_open) {
#pragma unroll
        for (int k = 0; k < L::Q; ++k) {
            const R gk = S::load(ld(src + (size_t)k * p.N, cell), inv_scale);
            rho_b += gk;
            jbx += R(L::cx[k]) * gk;
            jby += R(L::cy[k]) * gk;
            jbz += R(L::cz[k]) * gk;
        }
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
        int s[3];
        int open_axis = -1, open_side = 0;
        for (int a = 0; a < 3; ++a) {
            s[a] = X[a] - c[a];
            if (s[a] < 0) {
                if (p.bc_lo[a] == 0) s[a] += n[a];
                else if (open_axis < 0) { open_axis = a; open_side = -1; }
            } else if (s[a] >= n[a]) {
                if (p.bc_hi[a] == 0) s[a] -= n[a];
                else if (open_axis < 0) { open_axis = a; open_side = 1; }
            }
        }
        if (in_wall_layer(p, s[0], s[1], s[2])) {
            g[i] = S::load(ld(src + (size_t)opposite(i) * p.N, cell), inv_scale);
        } else if (open_axis < 0) {
            const uint32_t off = (uint32_t)s[0] + (uint32_t)p.nx * ((uint32_t)s[1] + (uint32_t)p.ny * (uint32_t)s[2]);
            g[i] = S::load(ld(src + (size_t)i * p.N, off), inv_scale);
        } else {
            const int kind = open_side < 0 ? p.bc_lo[open_axis] : p.bc_hi[open_axis];
            if (kind == 2) {
                g[i] = feq_shifted<L, R>(i, rho_b, R(p.rho0), R(p.inlet_u[0]), R(p.inlet_u[1]),
                                         R(p.inlet_u[2]));
            } else {
                const R inv = R(1) / rho_b;
                g[i] = feq_shifted<L, R>(i, R(p.outlet_rho), R(p.rho0), jbx * inv, jby * inv,
                                         jbz * inv);
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// The sweep.  One step: pull, moments, shift, equilibrium, relax + force,
// store into the other buffer.
// ---------------------------------------------------------------------------
template <class L, class S, int BC>
__global__ __launch_bounds__(1024) void sweep_kernel(const typename S::T* __restrict__ src,
                                                      typename S::T* __restrict__ dst,
                                                      const typename S::D* __restrict__ dfield,
                                                      Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const R inv_scale = R(p.inv_scale), scale = R(p.scale);
    R g[L::Q];
    if (BC == BC_PERIODIC) {
        gather_periodic<L, S>(src, p, x, y, z, inv_scale, g);
    } else {
        if (!gather_general<L, S>(src, p, (int)x, (int)y, (int)z, inv_scale, g)) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i) st(dst + (size_t)i * p.N, cell, S::store(R(0), scale));
            return;
        }
    }
    const R d = S::load_d(ld(dfield, cell));
    R drho, ux, uy, uz;
    collide<L, R>(g, d, R(p.F[0]), R(p.F[1]), R(p.F[2]), R(p.rho0), R(p.omega), R(p.pref), drho,
                  ux, uy, uz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        st(dst + (size_t)i * p.N, cell, S::store(g[i], scale));
    }
}

// ---------------------------------------------------------------------------
// FP64 block reduction of 4 values (wavefront shuffle, then across waves in
// LDS).  Thread 0 writes the block's partials.  Fixed order -> deterministic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ void block_sum4(double a, double b, double c, double d, double* out)
{
    __shared__ double red[16][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane == 0) {
        red[wid][0] = a;
        red[wid][1] = b;
        red[wid][2] = c;
        red[wid][3] = d;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Moments at the current time level (gather + moments, no collision).
template <class L, class S, int BC, class O>
__global__ __launch_bounds__(1024) void moments_kernel(const typename S::T* __restrict__ src,
                                                        O* __restrict__ drho_out,
                                                        O* __restrict__ u_out,
                                                        double* __restrict__ partials, Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const R inv_scale = R(p.inv_scale);
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (x < (uint32_t)p.nx) {
        const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
        R g[L::Q];
        bool fluid = true;
        if (BC == BC_PERIODIC) gather_periodic<L, S>(src, p, x, y, z, inv_scale, g);
        else fluid = gather_general<L, S>(src, p, (int)x, (int)y, (int)z, inv_scale, g);
        R drho = R(0), ux = R(0), uy = R(0), uz = R(0);
        if (fluid) moments_of<L, R>(g, R(p.F[0]), R(p.F[1]), R(p.F[2]), R(p.rho0), drho, ux, uy, uz);
        if (drho_out) drho_out[cell] = O(drho);
        if (u_out) {
            u_out[cell] = O(ux);
            u_out[(size_t)p.N + cell] = O(uy);
            u_out[2 * (size_t)p.N + cell] = O(uz);
        }
        if (fluid) {
            const double rho = p.rho0 + (double)drho;
            m0 = (double)drho;
            m1 = rho * (double)ux;
            m2 = rho * (double)uy;
            m3 = rho * (double)uz;
        }
    }
    if (partials) {
        const uint32_t b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)b);
    }
}

// Second pass: one block sums the per-block partials in a fixed order.
__global__ __launch_bounds__(256) void reduce4_kernel(const double* __restrict__ partials,
                                                      uint32_t nblocks, double* __restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (uint32_t k = threadIdx.x; k < nblocks; k += blockDim.x) {
        a += partials[4 * (size_t)k + 0];
        b += partials[4 * (size_t)k + 1];
        c += partials[4 * (size_t)k + 2];
        d += partials[4 * (size_t)k + 3];
    }
    block_sum4(a, b, c, d, out);
}

// Porosity conversion with validation: d must be finite and in [0, 1].
template <class I, class O>
__global__ __launch_bounds__(256) void porosity_kernel(const I* __restrict__ in, O* __restrict__ out,
                                                       uint32_t n, int* __restrict__ block_flags)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (k < n) {
        const double v = (double)in[k];
        bad = !(v >= 0.0 && v <= 1.0);  // also catches NaN
        out[k] = O(in[k]);
    }
    const int any = __syncthreads_or(bad);
    if (threadIdx.x == 0) block_flags[blockIdx.x] = any;
}

__global__ __launch_bounds__(256) void flags_or_kernel(const int* __restrict__ flags, uint32_t n,
                                                       int* __restrict__ out)
{
    int any = 0;
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) any |= flags[k];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) out[0] = any;
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
                                    const void* dfield, int bx, hipStream_t s)
{
    const Launch l = cell_launch(p, bx);
    auto* a = static_cast<const typename S::T*>(src);
    auto* b = static_cast<typename S::T*>(dst);
    auto* d = static_cast<const typename S::D*>(dfield);
    if (bcmode == BC_PERIODIC)
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_PERIODIC>), l.grid, l.block, 0, s, a, b, d, p);
    else
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_GENERAL>), l.grid, l.block, 0, s, a, b, d, p);
    return hipGetLastError();
}

template <class L>
static hipError_t sweep_dispatch_store(int storage, int bcmode, const Params& p, const void* src,
                                       void* dst, const void* dfield, int bx, hipStream_t s)
{
    switch (storage) {
    case StoreF64::code: return sweep_dispatch_bc<L, StoreF64>(bcmode, p, src, dst, dfield, bx, s);
    case StoreF32::code: return sweep_dispatch_bc<L, StoreF32>(bcmode, p, src, dst, dfield, bx, s);
    case StoreF16S::code: return sweep_dispatch_bc<L, StoreF16S>(bcmode, p, src, dst, dfield, bx, s);
    case StoreBF16S::code: return sweep_dispatch_bc<L, StoreBF16S>(bcmode, p, src, dst, dfield, bx, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int q, int storage, int bcmode, const Params& p, const void* src, void* dst,
                        const void* dfield, int bx, hipStream_t s)
{
    if (q == 9) return sweep_dispatch_store<D2Q9>(storage, bcmode, p, src, dst, dfield, bx, s);
    if (q == 19) return sweep_dispatch_store<D3Q19>(storage, bcmode, p, src, dst, dfield, bx, s);
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

hipError_t launch_reduce4(const double* partials, uint32_t nblocks, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce4_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

template <class I>
static hipError_t porosity_dispatch_out(const void* in, int storage, void* out, uint32_t n,
                                        int* flags, hipStream_t s)
{
    const uint32_t nb = (n + 255) / 256;
    auto* src = static_cast<const I*>(in);
    if (storage == StoreF64::code)
        hipLaunchKernelGGL((porosity_kernel<I, double>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<double*>(out), n, flags);
    else if (storage == StoreF32::code)
        hipLaunchKernelGGL((porosity_kernel<I, float>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<float*>(out), n, flags);
    else
        hipLaunchKernelGGL((porosity_kernel<I, _Float16>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<_Float16*>(out), n, flags);
    return hipGetLastError();
}

hipError_t launch_porosity_convert(int in_dtype, const void* in, int storage, void* out, uint32_t n,
                                   int* block_flags, int* flag_out, hipStream_t s)
{
    hipError_t e;
    if (in_dtype == 0) e = porosity_dispatch_out<double>(in, storage, out, n, block_flags, s);
    else if (in_dtype == 1) e = porosity_dispatch_out<float>(in, storage, out, n, block_flags, s);
    else e = porosity_dispatch_out<_Float16>(in, storage, out, n, block_flags, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(flags_or_kernel, dim3(1), dim3(256), 0, s, block_flags, (n + 255) / 256,
                       flag_out);
    return hipGetLastError();
}

}  // namespace hlbm
