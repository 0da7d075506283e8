// Per-cell device code of the HLBM sweep: addressing, pull gathers, moments
// and the homogenized BGK collision.  Included by the kernels in sweep.hip.
#pragma once
#include <type_traits>

#include "hlbm_internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"

// Multiply-add fusion only inside one source expression.  The default lets the
// code generator fuse across expressions, and its choices then depend on the
// surrounding kernel; with this setting every kernel that runs the same cell
// code (the single-lattice sweep, the batched step and the persistent batch)
// rounds identically, so their results agree bit for bit.
#pragma clang fp contract(on)

namespace hlbm {

// Element `idx` of a population row addressed by a 32-bit byte offset from a
// uniform base.  The host guarantees N * sizeof(T) < 2^32 for the rows these
// helpers index: populations in their storage type, porosity rows (never wider
// than the storage element), and adjoint population rows and moment record
// rows (the adjoint's element type, checked when a tape is set).  The offset cannot
// wrap, and every access can use the scalar-base + 32-bit vector-offset form
// of global loads and stores.  Per-cell arrays that may be wider (the link
// mask under 16-bit storage, the adjoint's FP64 cotangents and gradient, FP64
// moments) are indexed with ordinary 64-bit pointer arithmetic instead.
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

// Store of a new population: nothing reads it again within the step, so it
// is written with the non-temporal hint (streamed past the caches).
template <class T>
__device__ __forceinline__ void st_stream(T* __restrict__ base, uint32_t idx, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)));
}

// Porosity shift policies: the equilibrium velocity u_eq from u.
//   ScalarShift : u_eq = (1 - d) u                     (Sec. 3.2, varpi = 1 - d)
//   TensorShift : u_eq = (I - D) u, D = nu tau K^{-1}  (tensor permeability K;
//                 the isotropic case of Sec. 3.2 is D = d I)
// eq() works in R, eq_d() in FP64 (for the exact post-collision momentum).
template <class R>
struct ScalarShift {
    R d;
    __device__ __forceinline__ void eq(R ux, R uy, R uz, R& ex, R& ey, R& ez) const
    {
        const R sh = R(1) - d;
        ex = sh * ux;
        ey = sh * uy;
        ez = sh * uz;
    }
    __device__ __forceinline__ void eq_d(double ux, double uy, double uz, double& ex, double& ey,
                                         double& ez) const
    {
        const double sh = 1.0 - (double)d;
        ex = sh * ux;
        ey = sh * uy;
        ez = sh * uz;
    }
};

template <class R>
struct TensorShift {
    R xx, yy, zz, xy, xz, yz;
    __device__ __forceinline__ void eq(R ux, R uy, R uz, R& ex, R& ey, R& ez) const
    {
        ex = ux - (xx * ux + xy * uy + xz * uz);
        ey = uy - (xy * ux + yy * uy + yz * uz);
        ez = uz - (xz * ux + yz * uy + zz * uz);
    }
    __device__ __forceinline__ void eq_d(double ux, double uy, double uz, double& ex, double& ey,
                                         double& ez) const
    {
        const double dxx = xx, dyy = yy, dzz = zz, dxy = xy, dxz = xz, dyz = yz;
        ex = ux - (dxx * ux + dxy * uy + dxz * uz);
        ey = uy - (dxy * ux + dyy * uy + dyz * uz);
        ez = uz - (dxz * ux + dyz * uy + dzz * uz);
    }
};

// ---------------------------------------------------------------------------
// Collision of one fluid cell in the arithmetic type R (Sec. 3.2: BGK toward
// the homogenized Maxwellian; the velocity argument is (1 - d) u, or (I - D) u
// for a tensor control, see the shift policies below).
//   rho = rho0 + sum g, j = sum c g, u = (j + F/2)/rho, u_eq = (1 - d) u
//   g_i <- g_i - omega (g_i - g^eq_i(rho, u_eq)) + S_i
//   g^eq_i = w_i [ drho + rho (3 c.u_eq + 9/2 (c.u_eq)^2 - 3/2 u_eq.u_eq) ]
//   S_i    = (1 - 1/(2 tau)) w_i [ 3 (c_i - u).F + 9 (c_i.u)(c_i.F) ]
//
// Precision.  Mass and momentum are conserved modes: a rounding error made
// in them is never damped and accumulates over a run.  Two such errors are
// removed here, whatever R is:
//   * the moment sums (over populations far larger than drho) are carried in
//     FP64, so they are exact to ~1e-16 of their terms;
//   * the collision keeps mass and changes momentum by exactly
//     -omega (j - rho u_eq) + (1 - 1/(2 tau)) F (balance laws of the
//     homogenized Maxwellian, Sec. 3.2).  In FP32 the weights 1/3, 1/18,
//     1/36 are not representable and the relaxed populations would carry
//     those moments with a systematic bias of ~1e-8 per step; after the
//     relaxation the rest population and the axis populations absorb the
//     difference to the exact moments (computed in FP64).  In exact
//     arithmetic this correction is zero.
// Returns drho and u (the reported moments) through the reference arguments.
// ---------------------------------------------------------------------------
// The same collision with the moment sums in R and no correction, for the
// 16-bit storage forms: their stored values carry ~2^-11 relative rounding, far
// above anything the FP64 sums would remove, and at half the bytes per cell the
// FP64 work would become the sweep's bottleneck.
template <class L, class R, class Shift>
__device__ __forceinline__ void collide_plain(R (&g)[L::Q], const Shift& shift, R F0, R F1, R F2,
                                              R rho0, R omega, R pref, R& drho_out, R& ux_out,
                                              R& uy_out, R& uz_out)
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
    const R ux = (jx + R(0.5) * F0) * inv_rho;
    const R uy = (jy + R(0.5) * F1) * inv_rho;
    const R uz = (jz + R(0.5) * F2) * inv_rho;
    R ex, ey, ez;
    shift.eq(ux, uy, uz, ex, ey, ez);
    const R uu = ex * ex + ey * ey + ez * ez;
    const R uF = ux * F0 + uy * F1 + uz * F2;
    const R base = s - R(1.5) * rho * uu;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const R cx = R(L::cx[i]), cy = R(L::cy[i]), cz = R(L::cz[i]);
        const R w = R(L::w[i]);
        const R ce = cx * ex + cy * ey + cz * ez;
        const R cu = cx * ux + cy * uy + cz * uz;
        const R cF = cx * F0 + cy * F1 + cz * F2;
        const R geq = w * (base + rho * (R(3) * ce + R(4.5) * ce * ce));
        const R S = pref * w * (R(3) * (cF - uF) + R(9) * cu * cF);
        g[i] = g[i] + (S - omega * (g[i] - geq));
    }
    drho_out = s;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
}

// FP64 moments of the pre-collision populations gathered at one cell:
// s = sum g*, j = sum c g*, summed in population order.  The adjoint
// linearizes the collision at them; the forward sweep can record them.
struct Moms {
    double s, jx, jy, jz;
};

template <class L, class R, class Shift, bool Exact = true>
__device__ __forceinline__ void collide(R (&g)[L::Q], const Shift& shift, R F0, R F1, R F2, R rho0,
                                        R omega, R pref, R& drho_out, R& ux_out, R& uy_out, R& uz_out,
                                        Moms* sums = nullptr)
{
    if constexpr (!Exact) {
        collide_plain<L, R, Shift>(g, shift, F0, F1, F2, rho0, omega, pref, drho_out, ux_out, uy_out,
                                   uz_out);
        return;
    }
    double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double gi = (double)g[i];
        s += gi;
        if (L::cx[i]) jx += L::cx[i] > 0 ? gi : -gi;
        if (L::cy[i]) jy += L::cy[i] > 0 ? gi : -gi;
        if (L::cz[i]) jz += L::cz[i] > 0 ? gi : -gi;
    }
    const double rho_d = (double)rho0 + s;
    const double inv_rho_d = 1.0 / rho_d;
    const double uxd = (jx + 0.5 * (double)F0) * inv_rho_d;
    const double uyd = (jy + 0.5 * (double)F1) * inv_rho_d;
    const double uzd = (jz + 0.5 * (double)F2) * inv_rho_d;
    const R drho = R(s), rho = R(rho_d);
    const R ux = R(uxd), uy = R(uyd), uz = R(uzd);
    R ex, ey, ez;
    shift.eq(ux, uy, uz, ex, ey, ez);
    const R uu = ex * ex + ey * ey + ez * ez;
    const R uF = ux * F0 + uy * F1 + uz * F2;
    const R base = drho - R(1.5) * rho * uu;  // common part of every g^eq_i / w_i
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const R cx = R(L::cx[i]), cy = R(L::cy[i]), cz = R(L::cz[i]);
        const R w = R(L::w[i]);
        const R ce = cx * ex + cy * ey + cz * ez;
        const R cu = cx * ux + cy * uy + cz * uz;
        const R cF = cx * F0 + cy * F1 + cz * F2;
        const R geq = w * (base + rho * (R(3) * ce + R(4.5) * ce * ce));
        const R S = pref * w * (R(3) * (cF - uF) + R(9) * cu * cF);
        g[i] = g[i] + (S - omega * (g[i] - geq));
        const double gi = (double)g[i];
        m += gi;
        if (L::cx[i]) px += L::cx[i] > 0 ? gi : -gi;
        if (L::cy[i]) py += L::cy[i] > 0 ? gi : -gi;
        if (L::cz[i]) pz += L::cz[i] > 0 ? gi : -gi;
    }
    // exact post-collision moments from the pre-collision ones (FP64)
    const double om = (double)omega, pr = (double)pref;
    double exd, eyd, ezd;
    shift.eq_d(uxd, uyd, uzd, exd, eyd, ezd);
    const double tx = (1.0 - om) * jx + om * rho_d * exd + pr * (double)F0;
    const double ty = (1.0 - om) * jy + om * rho_d * eyd + pr * (double)F1;
    const double tz = (1.0 - om) * jz + om * rho_d * ezd + pr * (double)F2;
    constexpr int xp = axis_velocity<L>(0, 1), xm = axis_velocity<L>(0, -1);
    constexpr int yp = axis_velocity<L>(1, 1), ym = axis_velocity<L>(1, -1);
    const R hx = R(0.5 * (tx - px)), hy = R(0.5 * (ty - py));
    g[xp] += hx;
    g[xm] -= hx;
    g[yp] += hy;
    g[ym] -= hy;
    if (L::DIM == 3) {
        constexpr int zp = axis_velocity<L>(2, 1), zm = axis_velocity<L>(2, -1);
        const R hz = R(0.5 * (tz - pz));
        g[zp] += hz;
        g[zm] -= hz;
    }
    g[0] += R(s - m);
    drho_out = drho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
    // the FP64 pre-collision moment sums, as moments_f64 forms them (the
    // same sums in the same order)
    if (sums) *sums = Moms{s, jx, jy, jz};
}

// Moments only (no collision), same definitions as in collide().
// The sums run as the collision's do (FP64, rounded to R once; or in R for
// the 16-bit forms), so reported moments equal the collision's own.
template <class L, class R, bool Exact = true>
__device__ __forceinline__ void moments_of(const R (&g)[L::Q], R F0, R F1, R F2, R rho0, R& drho,
                                           R& ux, R& uy, R& uz)
{
    if constexpr (!Exact) {
        R s = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            s += g[i];
            if (L::cx[i]) jx += L::cx[i] > 0 ? g[i] : -g[i];
            if (L::cy[i]) jy += L::cy[i] > 0 ? g[i] : -g[i];
            if (L::cz[i]) jz += L::cz[i] > 0 ? g[i] : -g[i];
        }
        const R inv_rho = R(1) / (rho0 + s);
        drho = s;
        ux = (jx + R(0.5) * F0) * inv_rho;
        uy = (jy + R(0.5) * F1) * inv_rho;
        uz = (jz + R(0.5) * F2) * inv_rho;
        return;
    }
    double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double gi = (double)g[i];
        s += gi;
        if (L::cx[i]) jx += L::cx[i] > 0 ? gi : -gi;
        if (L::cy[i]) jy += L::cy[i] > 0 ? gi : -gi;
        if (L::cz[i]) jz += L::cz[i] > 0 ? gi : -gi;
    }
    const double inv_rho = 1.0 / ((double)rho0 + s);
    drho = R(s);
    ux = R((jx + 0.5 * (double)F0) * inv_rho);
    uy = R((jy + 0.5 * (double)F1) * inv_rho);
    uz = R((jz + 0.5 * (double)F2) * inv_rho);
}


template <class L, class R>
__device__ __forceinline__ Moms moments_f64(const R (&g)[L::Q])
{
    Moms m{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double gi = (double)g[i];
        m.s += gi;
        if (L::cx[i]) m.jx += L::cx[i] > 0 ? gi : -gi;
        if (L::cy[i]) m.jy += L::cy[i] > 0 ? gi : -gi;
        if (L::cz[i]) m.jz += L::cz[i] > 0 ? gi : -gi;
    }
    return m;
}

// Precision of the adjoint: FP64 for the FP64 form, FP32 for the others.  The
// adjoint populations, the reverse step's arithmetic and the moment record
// take it.
template <class S>
using AdjReal = typename std::conditional<std::is_same<S, StoreF64>::value, double, float>::type;

// Moment record of one forward step: four rows of N values in the adjoint's
// precision T (s, jx, jy, jz, rounded from the FP64 sums; cell index
// x + nx(y + ny z)).  The four rows together can pass 4 GiB, one row cannot
// (it has the element type and length of an adjoint population row, which
// hlbm_set_tape bounds): each row's start is formed in 64 bits and the cell's
// offset within it in 32.
template <class T>
__device__ __forceinline__ void record_moments(T* __restrict__ rec, uint32_t N, uint32_t cell, const Moms& m)
{
    const double v[4] = {m.s, m.jx, m.jy, m.jz};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T* const row = rec + (size_t)k * N;
        st(row, cell, T(v[k]));
    }
}

template <class T>
__device__ __forceinline__ Moms recorded_moments(const T* __restrict__ rec, uint32_t N, uint32_t cell)
{
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T* const row = rec + (size_t)k * N;
        v[k] = double(ld(row, cell));
    }
    return Moms{v[0], v[1], v[2], v[3]};
}

// ---------------------------------------------------------------------------
// Pull gather, fully periodic box: g*_i(x) = g_i(x - c_i) with wrap.  The box
// starts at cell `base` of the population rows (0 for a single lattice).  In
// all gathers below, population row i starts P elements after row i - 1
// (the row pitch: N cells plus the row pad).
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ void gather_periodic(const typename S::T* __restrict__ src, uint32_t P,
                                                uint32_t base, uint32_t nx, uint32_t ny, uint32_t nz,
                                                uint32_t x, uint32_t y, uint32_t z,
                                                typename S::R inv_scale, typename S::R (&g)[L::Q])
{
    // Source coordinate for c = -1, 0, +1 (index c + 1): x - c with wrap.
    const uint32_t xs[3] = {x + 1 == nx ? 0u : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const uint32_t off = base + xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        g[i] = S::load(ld(src + (size_t)i * P, off), inv_scale);
    }
}

// AA pattern, even step: the cell's own slots hold its pulled populations.
template <class L, class S>
__device__ __forceinline__ void gather_aa_even(const typename S::T* src, uint32_t P, uint32_t cell,
                                               typename S::R inv_scale, typename S::R (&g)[L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) g[i] = S::load(ld(src + (size_t)i * P, cell), inv_scale);
}

// AA pattern, odd step: population i arrives from slot opp(i) of x - c_i
// (where the even step left the post-collision population i), with wrap.
template <class L, class S>
__device__ __forceinline__ void gather_aa_odd(const typename S::T* src, uint32_t P, uint32_t nx, uint32_t ny,
                                              uint32_t nz, uint32_t x, uint32_t y, uint32_t z,
                                              typename S::R inv_scale, typename S::R (&g)[L::Q])
{
    const uint32_t xs[3] = {x + 1 == nx ? 0u : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const uint32_t off = xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
        g[i] = S::load(ld(src + (size_t)opposite(i) * P, off), inv_scale);
    }
}

// Select between two values.  Arguments are taken by value so the choice is a
// select of register values: a conditional over two lvalues would select
// between their addresses, which keeps the operands in private memory.
template <class T>
__device__ __forceinline__ T sel(bool c, T a, T b)
{
    return c ? a : b;
}

// Box geometry and face kinds as plain values.  Kernels copy these out of the
// launch parameters on entry; device code never indexes the parameter block
// through a pointer (which lets every boundary branch keep its operands in
// registers).
struct Box {
    int nx, ny, nz;
    int lo0, hi0, lo1, hi1, lo2, hi2;  // face kinds: 0 periodic, 1 wall, 2 inlet, 3 outlet
};

__device__ __forceinline__ Box box_of(const Params& p)
{
    Box b;
    b.nx = p.nx; b.ny = p.ny; b.nz = p.nz;
    b.lo0 = p.bc_lo[0]; b.hi0 = p.bc_hi[0];
    b.lo1 = p.bc_lo[1]; b.hi1 = p.bc_hi[1];
    b.lo2 = p.bc_lo[2]; b.hi2 = p.bc_hi[2];
    return b;
}

// A wall face makes its first (lo) or last (hi) layer of cells solid.
// Bitwise operators keep this a straight-line predicate (no short-circuit
// branches).
__device__ __forceinline__ bool in_wall_layer(const Box& b, int sx, int sy, int sz)
{
    const int w = ((b.lo0 == 1) & (sx == 0)) | ((b.hi0 == 1) & (sx == b.nx - 1)) |
                  ((b.lo1 == 1) & (sy == 0)) | ((b.hi1 == 1) & (sy == b.ny - 1)) |
                  ((b.lo2 == 1) & (sz == 0)) | ((b.hi2 == 1) & (sz == b.nz - 1));
    return w != 0;
}

// Source coordinate along one axis, s = X - c, wrapped when the axis is
// periodic (periodic faces come in pairs).  Written with selects only.
__device__ __forceinline__ int wrap_source(int X, int c, int n, bool periodic)
{
    const int s = X - c;
    const int w = sel(s < 0, s + n, sel(s >= n, s - n, s));
    return sel(periodic, w, s);
}

// Shifted second-order equilibrium of one population (open faces only).
template <class L, class R>
__device__ __forceinline__ R feq_shifted(int i, R rho, R rho0, R ux, R uy, R uz)
{
    const R cu = R(L::cx[i]) * ux + R(L::cy[i]) * uy + R(L::cz[i]) * uz;
    const R uu = ux * ux + uy * uy + uz * uz;
    return R(L::w[i]) * ((rho - rho0) + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
}

// Values an open face needs (copied from the launch parameters on entry).
template <class R>
struct OpenFaces {
    R rho0, in_ux, in_uy, in_uz, out_rho;
};

// Own post-collision density and velocity j_b/rho_b of a cell (what an open
// face's equilibrium is built from).
template <class L, class S>
__device__ __forceinline__ void own_state(const typename S::T* __restrict__ src, uint32_t P, uint32_t cell,
                                          typename S::R rho0, typename S::R inv_scale, typename S::R& rho_b,
                                          typename S::R& ubx, typename S::R& uby, typename S::R& ubz)
{
    using R = typename S::R;
    R r = rho0, jbx = R(0), jby = R(0), jbz = R(0);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const R gk = S::load(ld(src + (size_t)k * P, cell), inv_scale);
        r += gk;
        if (L::cx[k]) jbx += L::cx[k] > 0 ? gk : -gk;
        if (L::cy[k]) jby += L::cy[k] > 0 ? gk : -gk;
        if (L::cz[k]) jbz += L::cz[k] > 0 ? gk : -gk;
    }
    const R inv_b = R(1) / r;
    rho_b = r;
    ubx = jbx * inv_b;
    uby = jby * inv_b;
    ubz = jbz * inv_b;
}

// The x ends of a plain row, after its periodic gather: each direction whose
// pull crosses an x face (c_x = +1 at the lo end cell, -1 at the hi end cell)
// takes that face's rule in place of the wrapped value: from a wall layer,
// halfway bounce-back (this cell's opposite population); across an open face,
// the equilibrium from this cell's own post-collision state.  Only the end
// lanes of a row take the branch; they load this cell's own populations once
// (every load stays at this cell).
template <class L, class S>
__device__ __forceinline__ void fix_x_ends(const typename S::T* __restrict__ src, uint32_t P, const Box& b,
                                           const OpenFaces<typename S::R>& of, int x, uint32_t cell,
                                           typename S::R inv_scale, typename S::R (&g)[L::Q])
{
    using R = typename S::R;
    const bool at_lo = x == x_end_lo(b.lo0), at_hi = x == x_end_hi(b.hi0, b.nx);
    if (!(at_lo | at_hi)) return;
    R own[L::Q];
#pragma unroll
    for (int k = 0; k < L::Q; ++k) own[k] = S::load(ld(src + (size_t)k * P, cell), inv_scale);
    // own post-collision state, summed as own_state does
    R rho_b = of.rho0, jbx = R(0), jby = R(0), jbz = R(0);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        rho_b += own[k];
        if (L::cx[k]) jbx += L::cx[k] > 0 ? own[k] : -own[k];
        if (L::cy[k]) jby += L::cy[k] > 0 ? own[k] : -own[k];
        if (L::cz[k]) jbz += L::cz[k] > 0 ? own[k] : -own[k];
    }
    const R inv_b = R(1) / rho_b;
    const R ubx = jbx * inv_b, uby = jby * inv_b, ubz = jbz * inv_b;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        if (L::cx[i] == 0) continue;
        const bool hit = L::cx[i] > 0 ? at_lo : at_hi;
        const int kind = L::cx[i] > 0 ? b.lo0 : b.hi0;
        const bool inlet = kind == 2;
        const R e_rho = sel(inlet, rho_b, of.out_rho);
        const R e_ux = sel(inlet, of.in_ux, ubx);
        const R e_uy = sel(inlet, of.in_uy, uby);
        const R e_uz = sel(inlet, of.in_uz, ubz);
        const R eq = feq_shifted<L, R>(i, e_rho, of.rho0, e_ux, e_uy, e_uz);
        g[i] = sel(hit, sel(kind == 1, own[opposite(i)], eq), g[i]);
    }
}

// Pull gather of a cell on a plain row (see plain_row): the periodic gather,
// then the row's x ends.  Loads what gather_general would, value for value.
template <class L, class S>
__device__ __forceinline__ void gather_plain_row(const typename S::T* __restrict__ src, uint32_t P, const Box& b,
                                                 const OpenFaces<typename S::R>& of, int x, int y, int z,
                                                 typename S::R inv_scale, typename S::R (&g)[L::Q])
{
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    gather_periodic<L, S>(src, P, 0u, (uint32_t)b.nx, (uint32_t)b.ny, (uint32_t)b.nz, (uint32_t)x, (uint32_t)y,
                          (uint32_t)z, inv_scale, g);
    fix_x_ends<L, S>(src, P, b, of, x, cell, inv_scale, g);
}

// ---------------------------------------------------------------------------
// Pull gather with walls and open faces (the general rule).  The loads of a
// direction are straight-line selects: every address stays inside the box.
// A solid cell (wall layer), whose result the caller discards, loads nothing,
// and the cell's own state is loaded only where a source lies beyond an open
// face; both are branches on the cell's own classification.  The sweep
// kernels use it on the rows next to a y or z face and gather_plain_row on
// the others (a choice per row).  Per direction:
//   * periodic axes wrap;
//   * a source in a wall layer -> halfway bounce-back g*_i(x) = g_opp(i)(x)
//     (takes precedence on edges): the load address switches to this cell's
//     opposite population;
//   * a source beyond an open face (lowest axis first) -> equilibrium from the
//     cell's own post-collision state: inlet f^eq(rho_b, u_in), outlet
//     f^eq(rho_out, j_b/rho_b), shifted by w rho0; the load address switches
//     to this cell (always in bounds) and the value is replaced.
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ void gather_general(const typename S::T* __restrict__ src, uint32_t P,
                                               const Box& b, const OpenFaces<typename S::R>& of,
                                               int x, int y, int z, typename S::R inv_scale,
                                               typename S::R (&g)[L::Q])
{
    using R = typename S::R;
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    const bool px = b.lo0 == 0, py = b.lo1 == 0, pz = b.lo2 == 0;
    // Where the source of direction i lies: in the box, in a wall layer or
    // beyond a face (then that face's kind).
    auto source = [&](int i, bool& wall, bool& outside, int& kind, uint32_t& noff) {
        const int sx = wrap_source(x, L::cx[i], b.nx, px);
        const int sy = wrap_source(y, L::cy[i], b.ny, py);
        const int sz = wrap_source(z, L::cz[i], b.nz, pz);
        wall = in_wall_layer(b, sx, sy, sz);
        const bool out_x = (sx < 0) | (sx >= b.nx);
        const bool out_y = (sy < 0) | (sy >= b.ny);
        const bool out_z = (sz < 0) | (sz >= b.nz);
        outside = out_x | out_y | out_z;
        noff = (uint32_t)sx + (uint32_t)b.nx * ((uint32_t)sy + (uint32_t)b.ny * (uint32_t)sz);
        const int kx = sel(sx < 0, b.lo0, b.hi0);
        const int ky = sel(sy < 0, b.lo1, b.hi1);
        const int kz = sel(sz < 0, b.lo2, b.hi2);
        kind = sel(out_x, kx, sel(out_y, ky, kz));
    };
#pragma unroll
    for (int i = 0; i < L::Q; ++i) g[i] = R(0);
    // A cell in a wall layer is solid: every caller discards its result, so
    // it loads nothing (two branches in all, on the cell's own classification).
    if (in_wall_layer(b, x, y, z)) return;
    // this cell's own post-collision state, loaded only where a source lies
    // beyond an open face (the only use of it)
    bool open_face = false;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        bool wall, outside;
        int kind;
        uint32_t noff;
        source(i, wall, outside, kind, noff);
        open_face |= outside & !wall;
    }
    R rho_b = of.rho0, ubx = R(0), uby = R(0), ubz = R(0);
    if (open_face) own_state<L, S>(src, P, cell, of.rho0, inv_scale, rho_b, ubx, uby, ubz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        bool wall, outside;
        int kind;
        uint32_t noff;
        source(i, wall, outside, kind, noff);
        const uint32_t row = sel(wall, (uint32_t)opposite(i), (uint32_t)i);
        const uint32_t off = sel(wall | outside, cell, noff);
        const R loaded = S::load(ld(src + (size_t)row * P, off), inv_scale);
        const bool inlet = kind == 2;
        const R e_rho = sel(inlet, rho_b, of.out_rho);
        const R e_ux = sel(inlet, of.in_ux, ubx);
        const R e_uy = sel(inlet, of.in_uy, uby);
        const R e_uz = sel(inlet, of.in_uz, ubz);
        const R eq = feq_shifted<L, R>(i, e_rho, of.rho0, e_ux, e_uy, e_uz);
        g[i] = sel(outside & !wall, eq, loaded);
    }
}

// ---------------------------------------------------------------------------
// AA pattern with wall faces, odd step: population i from slot opp(i) of
// x - c_i, or from this cell's own slot i where x - c_i is solid (halfway
// bounce-back).  A fluid cell's sources stay inside the box (the wall layers
// belong to it); for a solid cell, whose result the caller discards, a source
// beyond the box also switches to the cell's own slot, so every address stays
// in bounds.
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ void gather_aa_odd_walls(const typename S::T* src, uint32_t P, const Box& b, int x,
                                                    int y, int z, typename S::R inv_scale,
                                                    typename S::R (&g)[L::Q])
{
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    const bool px = b.lo0 == 0, py = b.lo1 == 0, pz = b.lo2 == 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int sx = wrap_source(x, L::cx[i], b.nx, px);
        const int sy = wrap_source(y, L::cy[i], b.ny, py);
        const int sz = wrap_source(z, L::cz[i], b.nz, pz);
        const bool outside = (sx < 0) | (sx >= b.nx) | (sy < 0) | (sy >= b.ny) | (sz < 0) | (sz >= b.nz);
        const bool own = in_wall_layer(b, sx, sy, sz) | outside;
        const uint32_t noff = (uint32_t)sx + (uint32_t)b.nx * ((uint32_t)sy + (uint32_t)b.ny * (uint32_t)sz);
        const uint32_t row = sel(own, (uint32_t)i, (uint32_t)opposite(i));
        const uint32_t off = sel(own, cell, noff);
        g[i] = S::load(ld(src + (size_t)row * P, off), inv_scale);
    }
}

// Where the AA odd step with wall faces puts post-collision population i of
// (x, y, z): slot i of x + c_i, or this cell's own slot opp(i) where x + c_i
// is solid or beyond the box, or where the cell itself is solid: the row and
// the cell offset within it.
template <class L>
__device__ __forceinline__ void aa_odd_target_walls(const Box& b, int x, int y, int z, bool self_solid, int i,
                                                    uint32_t& row, uint32_t& off)
{
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    const bool px = b.lo0 == 0, py = b.lo1 == 0, pz = b.lo2 == 0;
    const int tx = wrap_source(x, -L::cx[i], b.nx, px);
    const int ty = wrap_source(y, -L::cy[i], b.ny, py);
    const int tz = wrap_source(z, -L::cz[i], b.nz, pz);
    const bool outside = (tx < 0) | (tx >= b.nx) | (ty < 0) | (ty >= b.ny) | (tz < 0) | (tz >= b.nz);
    const bool own = self_solid | in_wall_layer(b, tx, ty, tz) | outside;
    const uint32_t toff = (uint32_t)tx + (uint32_t)b.nx * ((uint32_t)ty + (uint32_t)b.ny * (uint32_t)tz);
    row = sel(own, (uint32_t)opposite(i), (uint32_t)i);
    off = sel(own, cell, toff);
}

// ---------------------------------------------------------------------------
// Pull gather in a periodic box with resolved solid cells: where the source of
// direction i is solid, halfway bounce-back g*_i(x) = g_opp(i)(x) (the link
// mask, precomputed per cell, says which sources are solid): the load address
// switches to this cell's opposite population.  Returns whether the cell
// itself is solid.  A solid cell's result is discarded by every caller (its
// populations are stored as zeros, its moments reported as zeros), so it
// loads nothing and gathers zeros: the one branch of this gather, which keeps
// the memory system to the fluid cells.  `base` offsets the box inside the
// population rows and the link mask (an item of a batch; 0 otherwise).
// ---------------------------------------------------------------------------
template <class L, class S>
__device__ __forceinline__ bool gather_masked(const typename S::T* __restrict__ src, uint32_t P,
                                              const uint32_t* __restrict__ linkmask, uint32_t base,
                                              uint32_t nx, uint32_t ny, uint32_t nz, uint32_t x,
                                              uint32_t y, uint32_t z, typename S::R inv_scale,
                                              typename S::R (&g)[L::Q])
{
    const uint32_t cell = base + x + nx * (y + ny * z);
    const uint32_t lm = linkmask[cell];  // 4 B per cell: may pass 4 GiB under 16-bit storage
    const bool solid = (lm & LINK_SOLID_SELF) != 0u;
    const uint32_t xs[3] = {x + 1 == nx ? 0u : x + 1, x, x == 0 ? nx - 1 : x - 1};
    const uint32_t ys[3] = {y + 1 == ny ? 0u : y + 1, y, y == 0 ? ny - 1 : y - 1};
    const uint32_t zs[3] = {z + 1 == nz ? 0u : z + 1, z, z == 0 ? nz - 1 : z - 1};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) g[i] = typename S::R(0);
    if (!solid) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const bool back = ((lm >> i) & 1u) != 0u;
            const uint32_t noff = base + xs[L::cx[i] + 1] + nx * (ys[L::cy[i] + 1] + ny * zs[L::cz[i] + 1]);
            const uint32_t row = sel(back, (uint32_t)opposite(i), (uint32_t)i);
            const uint32_t off = sel(back, cell, noff);
            g[i] = S::load(ld(src + (size_t)row * P, off), inv_scale);
        }
    }
    return solid;
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

}  // namespace hlbm
