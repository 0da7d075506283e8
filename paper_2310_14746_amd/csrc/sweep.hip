// Fused pull-stream + collide sweep of the homogenized lattice BGK scheme,
// moments gather, FP64 reductions and porosity conversion, for gfx950.
//
// Memory layout: structure of arrays, population i of cell c at
// buf[i*P + c], c = x + nx*(y + ny*z), rows P >= N elements apart (the
// pitch is padded past N; see row_pitch).  One thread owns one cell; a block
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
// src and dst are one buffer in the AA modes, so they carry no restrict here
// (the A/B kernels' own arguments do).
template <class L, class S, int BC, int PK, bool REC = false>
__device__ __forceinline__ bool sweep_cell(const typename S::T* src, typename S::T* dst,
                                           const typename S::D* __restrict__ dfield, const Params& p,
                                           uint32_t x, uint32_t y, uint32_t z, typename S::R& drho,
                                           typename S::R& ux, typename S::R& uy, typename S::R& uz,
                                           AdjReal<S>* __restrict__ rec = nullptr)
{
    using R = typename S::R;
    const uint32_t P = p.P;  // population rows, and the rows of a tensor control, are P elements apart
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const R inv_scale = R(p.inv_scale), scale = R(p.scale);
    const R F0 = R(p.F[0]), F1 = R(p.F[1]), F2 = R(p.F[2]);
    const R rho0 = R(p.rho0), omega = R(p.omega), pref = R(p.pref);
    // the porosity value is loaded before the gather, so that it is in flight
    // with the pulled populations (after the gather it would wait behind the
    // x-end lanes' branch on a plain row)
    const typename S::D d0 = ld(dfield, cell);
    R g[L::Q];
    bool solid = false;
    if (BC == BC_PERIODIC) {
        gather_periodic<L, S>(src, P, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
    } else if (BC == BC_AA_EVEN) {
        gather_aa_even<L, S>(src, P, cell, inv_scale, g);
    } else if (BC == BC_AA_ODD) {
        gather_aa_odd<L, S>(src, P, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
    } else if (BC == BC_AA_EVEN_W) {
        gather_aa_even<L, S>(src, P, cell, inv_scale, g);
        solid = in_wall_layer(box_of(p), (int)x, (int)y, (int)z);
    } else if (BC == BC_AA_ODD_W) {
        const Box b = box_of(p);
        gather_aa_odd_walls<L, S>(src, P, b, (int)x, (int)y, (int)z, inv_scale, g);
        solid = in_wall_layer(b, (int)x, (int)y, (int)z);
    } else if (BC == BC_MASKED) {
        solid = gather_masked<L, S>(src, P, p.linkmask, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
    } else if (BC == BC_PLAIN_ROW) {
        const Box b = box_of(p);
        const OpenFaces<R> of{rho0, R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                              R(p.outlet_rho)};
        gather_plain_row<L, S>(src, P, b, of, (int)x, (int)y, (int)z, inv_scale, g);
        solid = in_wall_layer(b, (int)x, (int)y, (int)z);
    } else {
        const Box b = box_of(p);
        const OpenFaces<R> of{rho0, R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                              R(p.outlet_rho)};
        gather_general<L, S>(src, P, b, of, (int)x, (int)y, (int)z, inv_scale, g);
        solid = in_wall_layer(b, (int)x, (int)y, (int)z);
    }
    // REC: the FP64 moments of the pulled populations, which the reverse
    // sweep linearizes the collision at, into this step's moment record.  The
    // forms with FP64 moment sums take them from the collision (the same sums);
    // the others sum them here.
    Moms sums;
    Moms* const want = (REC && S::exact_moments) ? &sums : nullptr;
    if (REC && !S::exact_moments) record_moments(rec, p.N, cell, moments_f64<L, R>(g));
    if (PK == PK_SCALAR) {
        const ScalarShift<R> sh{S::load_d(d0)};
        collide<L, R, decltype(sh), S::exact_moments>(g, sh, F0, F1, F2, rho0, omega, pref, drho, ux, uy, uz,
                                                      want);
    } else {
        // six rows xx, yy, zz, xy, xz, yz of the symmetric control D
        // (rows P apart, like the population rows)
        const TensorShift<R> sh{S::load_d(d0),
                                S::load_d(ld(dfield + (size_t)P, cell)),
                                S::load_d(ld(dfield + 2 * (size_t)P, cell)),
                                S::load_d(ld(dfield + 3 * (size_t)P, cell)),
                                S::load_d(ld(dfield + 4 * (size_t)P, cell)),
                                S::load_d(ld(dfield + 5 * (size_t)P, cell))};
        collide<L, R, decltype(sh), S::exact_moments>(g, sh, F0, F1, F2, rho0, omega, pref, drho, ux, uy, uz,
                                                      want);
    }
    if (REC && S::exact_moments) record_moments(rec, p.N, cell, sums);
    // The in-place steps use plain stores: the lines they write were read into
    // L2 by the same step, and there the non-temporal hint cost about 3% (FP32,
    // 512^3) where in the two-buffer sweep it gains about 2%.
    if (BC == BC_AA_EVEN || BC == BC_AA_EVEN_W) {
        // post-collision population i into this cell's slot opp(i); a solid
        // cell stores zeros there
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st(dst + (size_t)opposite(i) * P, cell, S::store(sel(solid, R(0), g[i]), scale));
    } else if (BC == BC_AA_ODD_W) {
        // post-collision population i into slot i of x + c_i, or into this
        // cell's own slot opp(i) where x + c_i is solid; a solid cell stores
        // zeros into its own slots
        const Box b = box_of(p);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            uint32_t row, off;
            aa_odd_target_walls<L>(b, (int)x, (int)y, (int)z, solid, i, row, off);
            st(dst + (size_t)row * P, off, S::store(sel(solid, R(0), g[i]), scale));
        }
    } else if (BC == BC_AA_ODD) {
        // post-collision population i into slot i of x + c_i
        const uint32_t nx = p.nx, ny = p.ny, nz = p.nz;
        const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0u : x + 1};
        const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0u : y + 1};
        const uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0u : z + 1};
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const uint32_t off = xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
            st(dst + (size_t)i * P, off, S::store(g[i], scale));
        }
    } else {
        // solid cells (wall layers, masked cells) hold zeros; selected, not branched
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st_stream(dst + (size_t)i * P, cell, S::store(sel(solid, R(0), g[i]), scale));
    }
    return solid;
}

// The row (y, z) of this block: (blockIdx.y, blockIdx.z), or with walls or
// open faces (BC_GENERAL) the row_of order (the rows that are not plain
// first).
template <int BC>
__device__ __forceinline__ void block_row(const Params& p, int& y, int& z)
{
    y = (int)blockIdx.y;
    z = (int)blockIdx.z;
    if (BC == BC_GENERAL)
        row_of((int)(blockIdx.y + gridDim.y * blockIdx.z), p.ny, p.nz, p.bc_lo[1], p.bc_hi[1], p.bc_lo[2],
               p.bc_hi[2], y, z);
}

// One cell x < nx of a sweep kernel on row (y, z) (from block_row).  With
// walls or open faces (BC_GENERAL) plain rows take gather_plain_row and the
// others the general rule: the choice is uniform per block, and each path
// keeps its own collision and stores.
template <class L, class S, int BC, int PK, bool REC = false>
__device__ __forceinline__ bool sweep_row_cell(const typename S::T* src, typename S::T* dst,
                                               const typename S::D* __restrict__ dfield, const Params& p,
                                               uint32_t x, int y, int z, typename S::R& drho, typename S::R& ux,
                                               typename S::R& uy, typename S::R& uz,
                                               AdjReal<S>* __restrict__ rec = nullptr)
{
    if (BC == BC_GENERAL && plain_row(y, z, p.ny, p.nz, p.bc_lo[1], p.bc_hi[1], p.bc_lo[2], p.bc_hi[2]))
        return sweep_cell<L, S, BC_PLAIN_ROW, PK, REC>(src, dst, dfield, p, x, (uint32_t)y, (uint32_t)z, drho, ux,
                                                       uy, uz, rec);
    return sweep_cell<L, S, BC, PK, REC>(src, dst, dfield, p, x, (uint32_t)y, (uint32_t)z, drho, ux, uy, uz, rec);
}

template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(1024) void sweep_kernel(const typename S::T* __restrict__ src,
                                                      typename S::T* __restrict__ dst,
                                                      const typename S::D* __restrict__ dfield,
                                                      Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    int y, z;
    block_row<BC>(p, y, z);
    R drho, ux, uy, uz;
    (void)sweep_row_cell<L, S, BC, PK>(src, dst, dfield, p, x, y, z, drho, ux, uy, uz);
}

// The same sweep on a step that an adjoint tape records: it also writes each
// cell's FP64 pre-collision moments (four rows of N doubles) to `rec`.
template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(1024) void sweep_record_kernel(const typename S::T* __restrict__ src,
                                                             typename S::T* __restrict__ dst,
                                                             const typename S::D* __restrict__ dfield,
                                                             AdjReal<S>* __restrict__ rec, Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    int y, z;
    block_row<BC>(p, y, z);
    R drho, ux, uy, uz;
    (void)sweep_row_cell<L, S, BC, PK, true>(src, dst, dfield, p, x, y, z, drho, ux, uy, uz, rec);
}

// In-place (AA) step: one buffer, even or odd mode.  Blocks of at most 256
// threads: the shifted form keeps 19 store addresses live beside the 19
// values, which in FP64 needs more than the 128 VGPRs a 1024-thread block
// leaves per lane.
template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(256) void sweep_aa_kernel(typename S::T* buf,
                                                         const typename S::D* __restrict__ dfield,
                                                         Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    R drho, ux, uy, uz;
    (void)sweep_cell<L, S, BC, PK>(buf, buf, dfield, p, x, blockIdx.y, blockIdx.z, drho, ux, uy, uz);
}

// The same step on a diagnostic step: the sweep also reduces the moments it
// has formed (time level of `src`, fluid cells) to FP64 block partials
// [sum drho, sum rho u_x, sum rho u_y, sum rho u_z], with the same block
// geometry and arithmetic as the moments kernel's totals.
template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(1024) void sweep_diag_kernel(const typename S::T* __restrict__ src,
                                                           typename S::T* __restrict__ dst,
                                                           const typename S::D* __restrict__ dfield,
                                                           double* __restrict__ partials, Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    int y, z;
    block_row<BC>(p, y, z);
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (x < (uint32_t)p.nx) {
        R drho, ux, uy, uz;
        const bool solid = sweep_row_cell<L, S, BC, PK>(src, dst, dfield, p, x, y, z, drho, ux, uy, uz);
        const double rho = p.rho0 + (double)drho;
        m0 = sel(solid, 0.0, (double)drho);
        m1 = sel(solid, 0.0, rho * (double)ux);
        m2 = sel(solid, 0.0, rho * (double)uy);
        m3 = sel(solid, 0.0, rho * (double)uz);
    }
    // the partial of the cells of row (y, z), x-block blockIdx.x, whatever
    // order the rows were taken in: the totals are summed in one order
    const uint32_t bk = blockIdx.x + gridDim.x * ((uint32_t)y + gridDim.y * (uint32_t)z);
    block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)bk);
}

template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(256) void sweep_aa_diag_kernel(typename S::T* buf,
                                                              const typename S::D* __restrict__ dfield,
                                                              double* __restrict__ partials, Params p)
{
    using R = typename S::R;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    if (x < (uint32_t)p.nx) {
        R drho, ux, uy, uz;
        const bool solid =
            sweep_cell<L, S, BC, PK>(buf, buf, dfield, p, x, blockIdx.y, blockIdx.z, drho, ux, uy, uz);
        const double rho = p.rho0 + (double)drho;
        m0 = sel(solid, 0.0, (double)drho);
        m1 = sel(solid, 0.0, rho * (double)ux);
        m2 = sel(solid, 0.0, rho * (double)uy);
        m3 = sel(solid, 0.0, rho * (double)uz);
    }
    const uint32_t bk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    block_sum4(m0, m1, m2, m3, partials + 4 * (size_t)bk);
}

// ---------------------------------------------------------------------------
// 16-bit storage, periodic box: two neighbouring cells of an x-row per
// thread.  A 16-bit row element is too narrow to keep the memory system busy
// one lane at a time; a pair is one 32-bit access per population.  The pair
// pulled for c_x = +1 starts one element to the left of the thread's own pair
// and the pair for c_x = -1 one to the right (2-byte aligned 32-bit loads);
// at the two ends of a row the pair wraps around, and the lane there patches
// the wrapped element with one more 16-bit load.  Each cell goes through the
// same collision as in sweep_kernel, so results are bit for bit those of the
// one-cell kernel.  Requires nx even and >= 4.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ uint32_t ld_pair(const typename S::T* __restrict__ row, uint32_t x)
{
    uint32_t w;
    __builtin_memcpy(&w, reinterpret_cast<const char*>(row) + x * (uint32_t)sizeof(typename S::T), 4);
    return w;
}

template <class S>
__device__ __forceinline__ typename S::R unpack(uint32_t bits16, typename S::R inv_scale)
{
    const uint16_t h = static_cast<uint16_t>(bits16);
    typename S::T v;
    __builtin_memcpy(&v, &h, 2);
    return S::load(v, inv_scale);
}

// The 16 bits of a stored element, in the low half of a word.
template <class S>
__device__ __forceinline__ uint32_t bits16(typename S::T v)
{
    uint16_t u;
    __builtin_memcpy(&u, &v, 2);
    return (uint32_t)u;
}

template <class S>
__global__ __launch_bounds__(1024) void sweep_pair_kernel(const typename S::T* __restrict__ src,
                                                           typename S::T* __restrict__ dst,
                                                           const typename S::D* __restrict__ dfield,
                                                           Params p)
{
    using L = D3Q19;
    using R = typename S::R;
    using T = typename S::T;
    const uint32_t x0 = 2u * (blockIdx.x * blockDim.x + threadIdx.x);
    const uint32_t nx = p.nx, ny = p.ny, nz = p.nz, P = p.P;
    if (x0 >= nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const R inv_scale = R(p.inv_scale), scale = R(p.scale);
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
    const bool first = x0 == 0, last = x0 + 2 == nx;
    const uint32_t cell = x0 + nx * (y + ny * z);
    // the two cells' controls as one 32-bit load (16-bit porosity elements),
    // issued before the gather: after it, it would wait behind the row-end
    // lanes' patches
    static_assert(sizeof(typename S::D) == 2, "pair kernel expects 16-bit porosity elements");
    uint32_t dw;
    __builtin_memcpy(&dw, reinterpret_cast<const char*>(dfield) + cell * 2u, 4);
    // Each population pair stays packed in one 32-bit word: the low cell is
    // unpacked, collided and its result written back into the low half, then
    // the same for the high cell.  Only one cell's 19 values are live as
    // floats at a time.
    uint32_t w[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const T* row = src + (size_t)i * P + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        // start of the pulled pair: x0 - c_x, kept inside the row at the ends
        uint32_t xs = x0;
        if (L::cx[i] > 0) xs = sel(first, x0, x0 - 1);
        if (L::cx[i] < 0) xs = sel(last, x0, x0 + 1);
        w[i] = ld_pair<S>(row, xs);
    }
    if (first) {  // c_x = +1 pulls (nx - 1, 0): the loaded pair was (0, 1)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (L::cx[i] <= 0) continue;
            const T* row = src + (size_t)i * P + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
            w[i] = bits16<S>(ld(row, nx - 1)) | (w[i] << 16);
        }
    }
    if (last) {  // c_x = -1 pulls (nx - 1, 0): the loaded pair was (nx - 2, nx - 1)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            if (L::cx[i] >= 0) continue;
            const T* row = src + (size_t)i * P + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
            w[i] = (w[i] >> 16) | (bits16<S>(ld(row, 0u)) << 16);
        }
    }
    const R F0 = R(p.F[0]), F1 = R(p.F[1]), F2 = R(p.F[2]);
    const R rho0 = R(p.rho0), omega = R(p.omega), pref = R(p.pref);
    R drho, ux, uy, uz;
    typename S::D d_lo, d_hi;
    const uint16_t dl = (uint16_t)(dw & 0xffffu), dh = (uint16_t)(dw >> 16);
    __builtin_memcpy(&d_lo, &dl, 2);
    __builtin_memcpy(&d_hi, &dh, 2);
    R g[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) g[i] = unpack<S>(w[i] & 0xffffu, inv_scale);
    collide<L, R, ScalarShift<R>, S::exact_moments>(g, ScalarShift<R>{S::load_d(d_lo)}, F0, F1, F2, rho0, omega,
                                                    pref, drho, ux, uy, uz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) w[i] = (w[i] & 0xffff0000u) | bits16<S>(S::store(g[i], scale));
#pragma unroll
    for (int i = 0; i < L::Q; ++i) g[i] = unpack<S>(w[i] >> 16, inv_scale);
    collide<L, R, ScalarShift<R>, S::exact_moments>(g, ScalarShift<R>{S::load_d(d_hi)}, F0, F1, F2, rho0, omega,
                                                    pref, drho, ux, uy, uz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        uint32_t* out = reinterpret_cast<uint32_t*>(dst + (size_t)i * P);
        st_stream(out, cell / 2u, (w[i] & 0xffffu) | (bits16<S>(S::store(g[i], scale)) << 16));
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
            gather_periodic<L, S>(src, p.P, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
        } else if (BC == BC_AA_EVEN) {
            gather_aa_even<L, S>(src, p.P, cell, inv_scale, g);
        } else if (BC == BC_AA_ODD) {
            gather_aa_odd<L, S>(src, p.P, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
        } else if (BC == BC_AA_EVEN_W) {
            gather_aa_even<L, S>(src, p.P, cell, inv_scale, g);
            fluid = !in_wall_layer(box_of(p), (int)x, (int)y, (int)z);
        } else if (BC == BC_AA_ODD_W) {
            const Box b = box_of(p);
            gather_aa_odd_walls<L, S>(src, p.P, b, (int)x, (int)y, (int)z, inv_scale, g);
            fluid = !in_wall_layer(b, (int)x, (int)y, (int)z);
        } else if (BC == BC_MASKED) {
            fluid = !gather_masked<L, S>(src, p.P, p.linkmask, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
        } else {
            const Box b = box_of(p);
            fluid = !in_wall_layer(b, (int)x, (int)y, (int)z);
            const OpenFaces<R> of{rho0, R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                                  R(p.outlet_rho)};
            gather_general<L, S>(src, p.P, b, of, (int)x, (int)y, (int)z, inv_scale, g);
        }
        R drho, ux, uy, uz;
        moments_of<L, R, S::exact_moments>(g, F0, F1, F2, rho0, drho, ux, uy, uz);
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

// Tensor control: six input rows (xx, yy, zz, xy, xz, yz) of N values; D must
// be symmetric with eigenvalues in [0, 1] (both D and I - D positive
// semidefinite: all principal minors >= 0, to a rounding allowance of 1e-12).
__device__ __forceinline__ bool psd3(double a, double b, double c, double ab, double ac, double bc)
{
    const double tol = -1e-12;
    const double m2ab = a * b - ab * ab, m2ac = a * c - ac * ac, m2bc = b * c - bc * bc;
    const double det = a * m2bc - ab * (ab * c - bc * ac) + ac * (ab * bc - b * ac);
    return (a >= tol) & (b >= tol) & (c >= tol) & (m2ab >= tol) & (m2ac >= tol) & (m2bc >= tol) &
           (det >= tol);
}

// The six output rows are `pitch` elements apart (the population row pitch).
template <class I, class O>
__global__ __launch_bounds__(256) void tensor_porosity_kernel(const I* __restrict__ in,
                                                              O* __restrict__ out, uint32_t n,
                                                              uint32_t pitch, int* __restrict__ flag)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (k < n) {
        double v[6];
        for (int r = 0; r < 6; ++r) {
            v[r] = (double)in[(size_t)r * n + k];
            bad |= !(v[r] == v[r]) | !(v[r] - v[r] == 0.0);  // NaN or infinite
            out[(size_t)r * pitch + k] = O(in[(size_t)r * n + k]);
        }
        const bool ok = psd3(v[0], v[1], v[2], v[3], v[4], v[5]) &&
                        psd3(1.0 - v[0], 1.0 - v[1], 1.0 - v[2], -v[3], -v[4], -v[5]);
        bad |= !ok;
    }
    const int any = __syncthreads_or(bad);
    if (threadIdx.x == 0 && any) atomicOr(flag, 1);
}

// AA-pattern state in A/B layout: out[i][x] = post-collision population i of
// cell x.  With odd_ready the buffer holds it in slot opp(i) of x; otherwise
// the buffer holds the pulled populations, and population i of x sits in slot
// i of x + c_i (periodic wrap), or, with wall faces, in slot opp(i) of x where
// x + c_i is solid or x itself is (whose slots hold zeros).  Raw element
// copies; the buffer's rows are P elements apart, the output's N.
template <class L, class E, bool OddReady, bool Walls>
__global__ __launch_bounds__(256) void aa_export_kernel(const E* __restrict__ buf, E* __restrict__ out, Box b,
                                                        uint32_t P)
{
    const uint32_t nx = b.nx, ny = b.ny, nz = b.nz;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const uint32_t N = nx * ny * nz;
    const uint32_t cell = x + nx * (y + ny * z);
    if (!OddReady && Walls) {
        const bool solid = in_wall_layer(b, (int)x, (int)y, (int)z);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            uint32_t row, off;
            aa_odd_target_walls<L>(b, (int)x, (int)y, (int)z, solid, i, row, off);
            out[(size_t)i * N + cell] = buf[(size_t)row * P + off];
        }
        return;
    }
    const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0u : x + 1};
    const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0u : y + 1};
    const uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0u : z + 1};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const uint32_t fwd = xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        out[(size_t)i * N + cell] = OddReady ? buf[(size_t)opposite(i) * P + cell] : buf[(size_t)i * P + fwd];
    }
}

// Link mask of a solid mask in a periodic box: bit i set where the pull
// source x - c_i of direction i is solid, bit 31 where x itself is.
template <class L>
__global__ __launch_bounds__(256) void linkmask_kernel(const unsigned char* __restrict__ mask,
                                                       uint32_t* __restrict__ linkmask, uint32_t nx,
                                                       uint32_t ny, uint32_t nz)
{
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const uint32_t cell = x + nx * (y + ny * z);
    const uint32_t xs[3] = {x + 1 == nx ? 0u : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
    uint32_t lm = mask[cell] ? LINK_SOLID_SELF : 0u;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const uint32_t src = xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        lm |= (mask[src] ? 1u : 0u) << i;
    }
    linkmask[cell] = lm;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
Launch cell_launch(const Params& p, int bx, int cells_per_thread)
{
    Launch l;
    const int tx = (p.nx + cells_per_thread - 1) / cells_per_thread;  // threads per x-row
    l.block = dim3(bx, 1, 1);
    l.grid = dim3((tx + bx - 1) / bx, p.ny, p.nz);
    l.nblocks = l.grid.x * l.grid.y * l.grid.z;
    return l;
}

template <class L, class S, int PK>
static hipError_t sweep_dispatch_bc(int bcmode, const Params& p, const void* src, void* dst,
                                    const void* dfield, int bx, hipStream_t s, double* diag, void* rec_v)
{
    auto* rec = static_cast<AdjReal<S>*>(rec_v);
    const Launch l = cell_launch(p, bx);
    auto* a = static_cast<const typename S::T*>(src);
    auto* b = static_cast<typename S::T*>(dst);
    auto* d = static_cast<const typename S::D*>(dfield);
    if (rec) {
        // recording steps of an adjoint tape: A/B, periodic or walls / open faces
        if (diag) return hipErrorInvalidValue;
        if (bcmode == BC_PERIODIC)
            hipLaunchKernelGGL((sweep_record_kernel<L, S, BC_PERIODIC, PK>), l.grid, l.block, 0, s, a, b, d, rec, p);
        else if (bcmode == BC_GENERAL)
            hipLaunchKernelGGL((sweep_record_kernel<L, S, BC_GENERAL, PK>), l.grid, l.block, 0, s, a, b, d, rec, p);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (bcmode == BC_AA_EVEN || bcmode == BC_AA_ODD || bcmode == BC_AA_EVEN_W || bcmode == BC_AA_ODD_W) {
        // one buffer: src and dst are the same address
        if (src != dst || bx > 256) return hipErrorInvalidValue;
        if (diag) {
            if (bcmode == BC_AA_EVEN)
                hipLaunchKernelGGL((sweep_aa_diag_kernel<L, S, BC_AA_EVEN, PK>), l.grid, l.block, 0, s, b, d, diag, p);
            else if (bcmode == BC_AA_ODD)
                hipLaunchKernelGGL((sweep_aa_diag_kernel<L, S, BC_AA_ODD, PK>), l.grid, l.block, 0, s, b, d, diag, p);
            else if (bcmode == BC_AA_EVEN_W)
                hipLaunchKernelGGL((sweep_aa_diag_kernel<L, S, BC_AA_EVEN_W, PK>), l.grid, l.block, 0, s, b, d, diag,
                                   p);
            else
                hipLaunchKernelGGL((sweep_aa_diag_kernel<L, S, BC_AA_ODD_W, PK>), l.grid, l.block, 0, s, b, d, diag,
                                   p);
        } else if (bcmode == BC_AA_EVEN) {
            hipLaunchKernelGGL((sweep_aa_kernel<L, S, BC_AA_EVEN, PK>), l.grid, l.block, 0, s, b, d, p);
        } else if (bcmode == BC_AA_ODD) {
            hipLaunchKernelGGL((sweep_aa_kernel<L, S, BC_AA_ODD, PK>), l.grid, l.block, 0, s, b, d, p);
        } else if (bcmode == BC_AA_EVEN_W) {
            hipLaunchKernelGGL((sweep_aa_kernel<L, S, BC_AA_EVEN_W, PK>), l.grid, l.block, 0, s, b, d, p);
        } else {
            hipLaunchKernelGGL((sweep_aa_kernel<L, S, BC_AA_ODD_W, PK>), l.grid, l.block, 0, s, b, d, p);
        }
        return hipGetLastError();
    }
    if (diag) {
        if (bcmode == BC_PERIODIC)
            hipLaunchKernelGGL((sweep_diag_kernel<L, S, BC_PERIODIC, PK>), l.grid, l.block, 0, s, a, b, d, diag, p);
        else if (bcmode == BC_MASKED)
            hipLaunchKernelGGL((sweep_diag_kernel<L, S, BC_MASKED, PK>), l.grid, l.block, 0, s, a, b, d, diag, p);
        else
            hipLaunchKernelGGL((sweep_diag_kernel<L, S, BC_GENERAL, PK>), l.grid, l.block, 0, s, a, b, d, diag, p);
    } else if (bcmode == BC_MASKED) {
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_MASKED, PK>), l.grid, l.block, 0, s, a, b, d, p);
    } else if (bcmode == BC_PERIODIC) {
        if constexpr (sizeof(typename S::T) == 2 && L::Q == 19 && PK == PK_SCALAR) {
            if (p.nx % 2 == 0 && p.nx >= 4) {
                const Launch lp = cell_launch(p, bx, 2);
                hipLaunchKernelGGL((sweep_pair_kernel<S>), lp.grid, lp.block, 0, s, a, b, d, p);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_PERIODIC, PK>), l.grid, l.block, 0, s, a, b, d, p);
    } else {
        // walls or open faces: plain rows and the general rule, chosen per row
        hipLaunchKernelGGL((sweep_kernel<L, S, BC_GENERAL, PK>), l.grid, l.block, 0, s, a, b, d, p);
    }
    return hipGetLastError();
}

template <class L, int PK>
static hipError_t sweep_dispatch_store(int storage, int bcmode, const Params& p, const void* src,
                                       void* dst, const void* dfield, int bx, hipStream_t s,
                                       double* diag, void* rec)
{
    switch (storage) {
    case StoreF64::code: return sweep_dispatch_bc<L, StoreF64, PK>(bcmode, p, src, dst, dfield, bx, s, diag, rec);
    case StoreF32::code: return sweep_dispatch_bc<L, StoreF32, PK>(bcmode, p, src, dst, dfield, bx, s, diag, rec);
    case StoreF16S::code: return sweep_dispatch_bc<L, StoreF16S, PK>(bcmode, p, src, dst, dfield, bx, s, diag, rec);
    case StoreBF16S::code:
        return sweep_dispatch_bc<L, StoreBF16S, PK>(bcmode, p, src, dst, dfield, bx, s, diag, rec);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int q, int storage, int bcmode, int pk, const Params& p, const void* src,
                        void* dst, const void* dfield, int bx, hipStream_t s, double* diag_partials,
                        void* moment_record)
{
    if (q == 9 && pk == PK_SCALAR)
        return sweep_dispatch_store<D2Q9, PK_SCALAR>(storage, bcmode, p, src, dst, dfield, bx, s, diag_partials,
                                                     moment_record);
    if (q == 19 && pk == PK_SCALAR)
        return sweep_dispatch_store<D3Q19, PK_SCALAR>(storage, bcmode, p, src, dst, dfield, bx, s, diag_partials,
                                                      moment_record);
    if (q == 19 && pk == PK_TENSOR)
        return sweep_dispatch_store<D3Q19, PK_TENSOR>(storage, bcmode, p, src, dst, dfield, bx, s, diag_partials,
                                                      moment_record);
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
    else if (bcmode == BC_AA_EVEN)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_AA_EVEN, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    else if (bcmode == BC_AA_ODD)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_AA_ODD, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    else if (bcmode == BC_AA_EVEN_W)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_AA_EVEN_W, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    else if (bcmode == BC_AA_ODD_W)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_AA_ODD_W, O>), l.grid, l.block, 0, s, a,
                           static_cast<O*>(drho), static_cast<O*>(u), partials, p);
    else if (bcmode == BC_MASKED)
        hipLaunchKernelGGL((moments_kernel<L, S, BC_MASKED, O>), l.grid, l.block, 0, s, a,
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

template <class L, class E>
static hipError_t aa_export_as(const Params& p, const void* buf, void* out, int odd_ready, hipStream_t s)
{
    const Launch l = cell_launch(p, 256);
    auto* a = static_cast<const E*>(buf);
    auto* b = static_cast<E*>(out);
    Box box;
    box.nx = p.nx; box.ny = p.ny; box.nz = p.nz;
    box.lo0 = p.bc_lo[0]; box.hi0 = p.bc_hi[0];
    box.lo1 = p.bc_lo[1]; box.hi1 = p.bc_hi[1];
    box.lo2 = p.bc_lo[2]; box.hi2 = p.bc_hi[2];
    const bool walls = (p.bc_lo[0] | p.bc_lo[1] | p.bc_lo[2] | p.bc_hi[0] | p.bc_hi[1] | p.bc_hi[2]) != 0;
    if (odd_ready)
        hipLaunchKernelGGL((aa_export_kernel<L, E, true, false>), l.grid, l.block, 0, s, a, b, box, p.P);
    else if (walls)
        hipLaunchKernelGGL((aa_export_kernel<L, E, false, true>), l.grid, l.block, 0, s, a, b, box, p.P);
    else
        hipLaunchKernelGGL((aa_export_kernel<L, E, false, false>), l.grid, l.block, 0, s, a, b, box, p.P);
    return hipGetLastError();
}

template <class L>
static hipError_t aa_export_elem(int storage, const Params& p, const void* buf, void* out, int odd_ready,
                                 hipStream_t s)
{
    if (storage == StoreF64::code) return aa_export_as<L, uint64_t>(p, buf, out, odd_ready, s);
    if (storage == StoreF32::code) return aa_export_as<L, uint32_t>(p, buf, out, odd_ready, s);
    if (storage == StoreF16S::code || storage == StoreBF16S::code)
        return aa_export_as<L, uint16_t>(p, buf, out, odd_ready, s);
    return hipErrorInvalidValue;
}

hipError_t launch_aa_export(int q, int storage, const Params& p, const void* buf, void* out, int odd_ready,
                            hipStream_t s)
{
    if (q == 9) return aa_export_elem<D2Q9>(storage, p, buf, out, odd_ready, s);
    if (q == 19) return aa_export_elem<D3Q19>(storage, p, buf, out, odd_ready, s);
    return hipErrorInvalidValue;
}

hipError_t launch_linkmask(int q, const Params& p, const unsigned char* mask, uint32_t* linkmask,
                           hipStream_t s)
{
    const Launch l = cell_launch(p, 256);
    if (q == 9)
        hipLaunchKernelGGL(linkmask_kernel<D2Q9>, l.grid, l.block, 0, s, mask, linkmask, (uint32_t)p.nx,
                           (uint32_t)p.ny, (uint32_t)p.nz);
    else
        hipLaunchKernelGGL(linkmask_kernel<D3Q19>, l.grid, l.block, 0, s, mask, linkmask, (uint32_t)p.nx,
                           (uint32_t)p.ny, (uint32_t)p.nz);
    return hipGetLastError();
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

template <class I>
static hipError_t tensor_dispatch_out(const void* in, int storage, void* out, uint32_t n, uint32_t pitch,
                                      int* flag, hipStream_t s)
{
    const uint32_t nb = (n + 255) / 256;
    auto* src = static_cast<const I*>(in);
    if (storage == StoreF64::code)
        hipLaunchKernelGGL((tensor_porosity_kernel<I, double>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<double*>(out), n, pitch, flag);
    else if (storage == StoreF32::code)
        hipLaunchKernelGGL((tensor_porosity_kernel<I, float>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<float*>(out), n, pitch, flag);
    else
        hipLaunchKernelGGL((tensor_porosity_kernel<I, _Float16>), dim3(nb), dim3(256), 0, s, src,
                           static_cast<_Float16*>(out), n, pitch, flag);
    return hipGetLastError();
}

hipError_t launch_porosity_convert(int in_dtype, const void* in, int storage, int pk, void* out,
                                   uint32_t n, uint32_t pitch, int* flag, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    if (pk == PK_TENSOR) {
        if (in_dtype == 0) return tensor_dispatch_out<double>(in, storage, out, n, pitch, flag, s);
        if (in_dtype == 1) return tensor_dispatch_out<float>(in, storage, out, n, pitch, flag, s);
        return tensor_dispatch_out<_Float16>(in, storage, out, n, pitch, flag, s);
    }
    if (in_dtype == 0) return porosity_dispatch_out<double>(in, storage, out, n, flag, s);
    if (in_dtype == 1) return porosity_dispatch_out<float>(in, storage, out, n, flag, s);
    return porosity_dispatch_out<_Float16>(in, storage, out, n, flag, s);
}

}  // namespace hlbm
