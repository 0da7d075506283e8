// Discrete adjoint of the sweep (reverse mode) for gradients of an objective
// of the moments with respect to the porosity control: d = 1 - varpi
// (Sec. 3.2), or the six rows xx, yy, zz, xy, xz, yz of a symmetric tensor D
// (u_eq = (I - D) u; an off-diagonal row is one variable at two places).
//
// One forward step is y_t = S(x_{t-1}) (pull streaming) followed by
// x_t = C(y_t, d) (the homogenized BGK collision of Sec. 3.2, cell-local), and
// the objective observes the moments M(S(x_T)).  The reverse sweep carries the
// adjoint of the pre-collision populations, lambda_t = dJ/dy_t:
//
//   lambda_{T+1} = M^T (dJ/drho, dJ/du)                         (seed kernel)
//   lambda_t     = C_y(y_t, d)^T S^T lambda_{t+1},
//   dJ/dd       += C_d(y_t, d)^T S^T lambda_{t+1}              (adjoint kernel)
//
// for t = T, T-1, ...  Both kernels are per-cell gathers with the sweep's
// launch geometry:
//   * S^T as a gather.  Pull streaming reads population k of cell x + c_k, so
//     its transpose reads the adjoint of population k at x + c_k.  Where the
//     forward rule at x for direction opp(k) bounced back, the transpose reads
//     this cell's own opp(k) adjoint; where it took an open-face equilibrium
//     built from this cell's post-collision state, the transpose adds that
//     equilibrium's derivative.  The classification per direction is the
//     forward gather's own (same helpers), with +c_k in place of -c_k.
//   * C^T by the chain rule through the moments: with A = sum_i pb_i g^eq_i
//     and B = sum_i pb_i S_i, the adjoint needs only the weighted moments
//     P0 = sum w pb, P1 = sum w c pb, P2 = sum w c c pb of the incoming adjoint
//     pb, not the 19x19 Jacobian.
//   * The collision is linearized at the FP64 moments (rho, j) of y_t, which
//     the recording forward sweep wrote to a moment record (four rows of N
//     doubles per step), so no forward population is read.  The
//     post-collision moments of this cell at step t, needed by the open-face
//     derivatives, follow from them by the collision's balance laws (mass
//     kept, momentum (1 - omega) j + omega rho u_eq + (1 - 1/(2 tau)) F).
//
// Layout: adjoint populations are rows lam[k*P + cell], P elements apart like
// the forward state's rows, FP64 for the FP64 form and FP32 for the others.
// The reverse step computes in that precision (the seed in FP64); dJ/dd is one
// FP64 value per cell and control row, and each step's contribution is added
// to it in FP64.  Blocks hold at most 256 threads (the reverse step needs more
// registers than a 1024-thread block leaves per thread); the launchers clamp
// the block width.
#include <type_traits>

#include "cell.hpp"

namespace hlbm {

// Element type of the adjoint populations (and of the moment record) for
// storage policy S.
template <class S>
using LamT = AdjReal<S>;

// Gather of the forward pre-collision populations y at (x, y, z) from the
// post-collision state `src`, reduced at once to FP64 moments.
template <class L, class S, int BC>
__device__ __forceinline__ Moms forward_moments(const typename S::T* __restrict__ src, const Params& p,
                                                uint32_t x, uint32_t y, uint32_t z)
{
    using R = typename S::R;
    const R inv_scale = R(p.inv_scale);
    R g[L::Q];
    if (BC == BC_PERIODIC) {
        gather_periodic<L, S>(src, p.P, 0u, p.nx, p.ny, p.nz, x, y, z, inv_scale, g);
    } else {
        const Box b = box_of(p);
        const OpenFaces<R> of{R(p.rho0), R(p.inlet_u[0]), R(p.inlet_u[1]), R(p.inlet_u[2]),
                              R(p.outlet_rho)};
        gather_general<L, S>(src, p.P, b, of, (int)x, (int)y, (int)z, inv_scale, g);
    }
    return moments_f64<L, R>(g);
}

// ---------------------------------------------------------------------------
// Seed: lambda_k = dJ/ddrho + sum_a dJ/du_a (c_ka - u_a)/rho at the moments'
// time level (drho = sum g, u = (j + F/2)/rho).  Solid cells get zeros.
// ---------------------------------------------------------------------------
template <class L, class S, int BC>
__global__ __launch_bounds__(256) void adjoint_seed_kernel(const typename S::T* __restrict__ src,
                                                            const double* __restrict__ drho_bar,
                                                            const double* __restrict__ u_bar,
                                                            LamT<S>* __restrict__ lam, Params p)
{
    const uint32_t N = p.N;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const Moms m = forward_moments<L, S, BC>(src, p, x, y, z);
    const double inv_rho = 1.0 / (p.rho0 + m.s);
    const double ux = (m.jx + 0.5 * p.F[0]) * inv_rho;
    const double uy = (m.jy + 0.5 * p.F[1]) * inv_rho;
    const double uz = (m.jz + 0.5 * p.F[2]) * inv_rho;
    // FP64 rows of N values can pass 4 GiB: 64-bit indexing
    const double rb = drho_bar[cell];
    const double bx = u_bar[cell] * inv_rho;
    const double by = u_bar[(size_t)N + cell] * inv_rho;
    const double bz = u_bar[2 * (size_t)N + cell] * inv_rho;
    const double base = rb - (bx * ux + by * uy + bz * uz);
    bool solid = false;
    if (BC != BC_PERIODIC) solid = in_wall_layer(box_of(p), (int)x, (int)y, (int)z);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const double v = base + double(L::cx[k]) * bx + double(L::cy[k]) * by + double(L::cz[k]) * bz;
        st(lam + (size_t)k * p.P, cell, LamT<S>(sel(solid, 0.0, v)));
    }
}

// ---------------------------------------------------------------------------
// S^T: adjoint of the post-collision populations of this cell from the
// adjoint of the next step's pre-collision populations.
// ---------------------------------------------------------------------------
template <class L, class A>
__device__ __forceinline__ void stream_adjoint_periodic(const A* __restrict__ lam, uint32_t P,
                                                        const Params& p, uint32_t x, uint32_t y,
                                                        uint32_t z, A (&pb)[L::Q])
{
    const uint32_t nx = p.nx, ny = p.ny, nz = p.nz;
    // x + c for c = -1, 0, +1 (index c + 1), wrapped
    const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0u : x + 1};
    const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0u : y + 1};
    const uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0u : z + 1};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const uint32_t off = xs[L::cx[k] + 1] + nx * (ys[L::cy[k] + 1] + ny * zs[L::cz[k] + 1]);
        pb[k] = ld(lam + (size_t)k * P, off);
    }
}

// Walls and open faces.  `rho_b`, (ubx, uby, ubz) are this cell's
// post-collision density and velocity j_b/rho_b at the forward step whose
// open-face equilibria are being differentiated.
template <class L, class A>
__device__ __forceinline__ void stream_adjoint_general(const A* __restrict__ lam, uint32_t P,
                                                       const Params& p, int x, int y, int z,
                                                       A rho_b, A ubx, A uby, A ubz, A (&pb)[L::Q])
{
    const Box b = box_of(p);
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    const bool px = b.lo0 == 0, py = b.lo1 == 0, pz = b.lo2 == 0;
    const A uix = A(p.inlet_u[0]), uiy = A(p.inlet_u[1]), uiz = A(p.inlet_u[2]);
    const A uin2 = uix * uix + uiy * uiy + uiz * uiz;
    const A rout = A(p.outlet_rho);
    A a_in = 0, bvx = 0, bvy = 0, bvz = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        // neighbour x + c_k = x - c_opp(k): the forward source of direction opp(k) at x
        const int sx = wrap_source(x, -L::cx[k], b.nx, px);
        const int sy = wrap_source(y, -L::cy[k], b.ny, py);
        const int sz = wrap_source(z, -L::cz[k], b.nz, pz);
        const bool wall = in_wall_layer(b, sx, sy, sz);
        const bool out_x = (sx < 0) | (sx >= b.nx);
        const bool out_y = (sy < 0) | (sy >= b.ny);
        const bool out_z = (sz < 0) | (sz >= b.nz);
        const bool outside = out_x | out_y | out_z;
        const bool own = wall | outside;
        const uint32_t noff = (uint32_t)sx + (uint32_t)b.nx * ((uint32_t)sy + (uint32_t)b.ny * (uint32_t)sz);
        const uint32_t row = sel(own, (uint32_t)opposite(k), (uint32_t)k);
        const uint32_t off = sel(own, cell, noff);
        const A v = ld(lam + (size_t)row * P, off);
        const bool open = outside & !wall;
        pb[k] = sel(open, A(0), v);
        // open face: v is the adjoint of this cell's pre-collision population
        // i = opp(k), which the forward step took from an equilibrium
        const int kx = sel(sx < 0, b.lo0, b.hi0);
        const int ky = sel(sy < 0, b.lo1, b.hi1);
        const int kz = sel(sz < 0, b.lo2, b.hi2);
        const int kind = sel(out_x, kx, sel(out_y, ky, kz));
        const bool inlet = kind == 2;
        const int i = opposite(k);
        const A w = A(L::w[i]);
        const A cix = A(L::cx[i]), ciy = A(L::cy[i]), ciz = A(L::cz[i]);
        const A cin = cix * uix + ciy * uiy + ciz * uiz;
        // inlet f^eq(rho_b, u_in): d/d rho_b
        const A d_in = w * (A(1) + A(3) * cin + A(4.5) * cin * cin - A(1.5) * uin2);
        a_in += sel(open & inlet, v * d_in, A(0));
        // outlet f^eq(rho_out, u_b): d/d u_b
        const A cub = cix * ubx + ciy * uby + ciz * ubz;
        const A wv = sel(open & !inlet, v * w * rout, A(0));
        bvx += wv * (A(3) * cix + A(9) * cub * cix - A(3) * ubx);
        bvy += wv * (A(3) * ciy + A(9) * cub * ciy - A(3) * uby);
        bvz += wv * (A(3) * ciz + A(9) * cub * ciz - A(3) * ubz);
    }
    // rho_b depends on every own population with weight 1, u_b = j_b/rho_b
    const A inv_b = A(1) / rho_b;
    const A common = a_in - (bvx * ubx + bvy * uby + bvz * ubz) * inv_b;
    const A gx = bvx * inv_b, gy = bvy * inv_b, gz = bvz * inv_b;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        pb[k] += common + A(L::cx[k]) * gx + A(L::cy[k]) * gy + A(L::cz[k]) * gz;
}

// The x ends of a plain row, after stream_adjoint_periodic: the transpose of
// fix_x_ends.  Direction k pulls from x + c_k, which crosses the lo face
// where c_x = -1 (at the lo end cell) and the hi face where c_x = +1 (at the
// hi end cell).  There the forward step took population opp(k) of this cell
// by bounce-back (wall: read this cell's adjoint of opp(k)) or from an open
// face's equilibrium (nothing from the neighbour; the equilibrium's
// derivatives, as in stream_adjoint_general).  Only the end lanes of a row
// call it; every load stays at this cell.
template <class L, class A>
__device__ __forceinline__ void stream_adjoint_x_ends(const A* __restrict__ lam, uint32_t P, const Params& p,
                                                      const Box& b, bool at_lo, bool at_hi, uint32_t cell,
                                                      A rho_b, A ubx, A uby, A ubz, A (&pb)[L::Q])
{
    const A uix = A(p.inlet_u[0]), uiy = A(p.inlet_u[1]), uiz = A(p.inlet_u[2]);
    const A uin2 = uix * uix + uiy * uiy + uiz * uiz;
    const A rout = A(p.outlet_rho);
    A a_in = 0, bvx = 0, bvy = 0, bvz = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        if (L::cx[k] == 0) continue;
        const bool hit = L::cx[k] < 0 ? at_lo : at_hi;
        const int kind = L::cx[k] < 0 ? b.lo0 : b.hi0;
        const A v = ld(lam + (size_t)opposite(k) * P, cell);
        const bool open = hit & (kind >= 2);
        pb[k] = sel(open, A(0), sel(hit, v, pb[k]));
        const bool inlet = kind == 2;
        const int i = opposite(k);
        const A w = A(L::w[i]);
        const A cix = A(L::cx[i]), ciy = A(L::cy[i]), ciz = A(L::cz[i]);
        const A cin = cix * uix + ciy * uiy + ciz * uiz;
        const A d_in = w * (A(1) + A(3) * cin + A(4.5) * cin * cin - A(1.5) * uin2);
        a_in += sel(open & inlet, v * d_in, A(0));
        const A cub = cix * ubx + ciy * uby + ciz * ubz;
        const A wv = sel(open & !inlet, v * w * rout, A(0));
        bvx += wv * (A(3) * cix + A(9) * cub * cix - A(3) * ubx);
        bvy += wv * (A(3) * ciy + A(9) * cub * ciy - A(3) * uby);
        bvz += wv * (A(3) * ciz + A(9) * cub * ciz - A(3) * ubz);
    }
    const A inv_b = A(1) / rho_b;
    const A common = a_in - (bvx * ubx + bvy * uby + bvz * ubz) * inv_b;
    const A gx = bvx * inv_b, gy = bvy * inv_b, gz = bvz * inv_b;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        pb[k] += common + A(L::cx[k]) * gx + A(L::cy[k]) * gy + A(L::cz[k]) * gz;
}

// ---------------------------------------------------------------------------
// The control in the adjoint's arithmetic A: u_eq = M u with M = (1 - d) I
// (scalar) or M = I - D (tensor; symmetric, so M^T = M).
//   om_m(om, a) = omega M a
//   grad(om, Av, u, g): g_r = omega Av . (dM/dtheta_r) u, the cotangent of
//   control row r, with dM/dd = -I for the scalar d, -e_a e_a^T for a
//   diagonal row and -(e_a e_b^T + e_b e_a^T) for an off-diagonal row (a, b).
// ---------------------------------------------------------------------------
template <class A>
struct AdjScalar {
    static constexpr int rows = 1;
    A d;
    template <class S>
    __device__ __forceinline__ static AdjScalar load(const typename S::D* __restrict__ f, uint32_t, uint32_t cell)
    {
        return AdjScalar{A(S::load_d(ld(f, cell)))};
    }
    __device__ __forceinline__ void eq(A ux, A uy, A uz, A& vx, A& vy, A& vz) const
    {
        const A sh = A(1) - d;
        vx = sh * ux;
        vy = sh * uy;
        vz = sh * uz;
    }
    __device__ __forceinline__ void om_m(A om, A ax, A ay, A az, A& bx, A& by, A& bz) const
    {
        const A s = om * (A(1) - d);
        bx = s * ax;
        by = s * ay;
        bz = s * az;
    }
    __device__ __forceinline__ void grad(A om, A Avx, A Avy, A Avz, A ux, A uy, A uz, A (&g)[1]) const
    {
        g[0] = -om * (Avx * ux + Avy * uy + Avz * uz);
    }
};

template <class A>
struct AdjTensor {
    static constexpr int rows = 6;
    A xx, yy, zz, xy, xz, yz;
    template <class S>
    __device__ __forceinline__ static AdjTensor load(const typename S::D* __restrict__ f, uint32_t pitch,
                                                     uint32_t cell)
    {
        return AdjTensor{A(S::load_d(ld(f, cell))),
                         A(S::load_d(ld(f + (size_t)pitch, cell))),
                         A(S::load_d(ld(f + 2 * (size_t)pitch, cell))),
                         A(S::load_d(ld(f + 3 * (size_t)pitch, cell))),
                         A(S::load_d(ld(f + 4 * (size_t)pitch, cell))),
                         A(S::load_d(ld(f + 5 * (size_t)pitch, cell)))};
    }
    __device__ __forceinline__ void eq(A ux, A uy, A uz, A& vx, A& vy, A& vz) const
    {
        vx = ux - (xx * ux + xy * uy + xz * uz);
        vy = uy - (xy * ux + yy * uy + yz * uz);
        vz = uz - (xz * ux + yz * uy + zz * uz);
    }
    __device__ __forceinline__ void om_m(A om, A ax, A ay, A az, A& bx, A& by, A& bz) const
    {
        A mx, my, mz;
        eq(ax, ay, az, mx, my, mz);
        bx = om * mx;
        by = om * my;
        bz = om * mz;
    }
    __device__ __forceinline__ void grad(A om, A Avx, A Avy, A Avz, A ux, A uy, A uz, A (&g)[6]) const
    {
        g[0] = -om * (Avx * ux);
        g[1] = -om * (Avy * uy);
        g[2] = -om * (Avz * uz);
        g[3] = -om * (Avx * uy + Avy * ux);
        g[4] = -om * (Avx * uz + Avz * ux);
        g[5] = -om * (Avy * uz + Avz * uy);
    }
};

template <int PK, class A>
using AdjShift = typename std::conditional<PK == PK_TENSOR, AdjTensor<A>, AdjScalar<A>>::type;

// ---------------------------------------------------------------------------
// C^T of one fluid cell.  In: the recorded moments of y, the control, and pb =
// adjoint of the post-collision populations.  Out: pb overwritten with the
// adjoint of the pre-collision populations, and this step's cotangent of each
// control row in g.
//   u = (j + F/2)/rho, v = M u
//   dA/drho = P0 (1 - 3/2 v.v) + 3 P1.v + 9/2 v.P2.v
//   dA/dv   = rho (3 P1 + 9 P2 v - 3 P0 v)
//   dB/du   = (1 - 1/(2 tau)) (9 P2 F - 3 P0 F)
//   ubar    = omega M^T dA/dv + dB/du
//   pre_k   = (1 - omega) pb_k + omega dA/drho - ubar.u/rho + c_k.ubar/rho
//   g_r     = omega dA/dv . (dM/dtheta_r) u
// ---------------------------------------------------------------------------
template <class L, class A, class Sh>
__device__ __forceinline__ void collide_adjoint(const Moms& m, const Sh& sh, const Params& p,
                                                A (&pb)[L::Q], A (&g)[Sh::rows])
{
    const A om = A(p.omega), pref = A(p.pref);
    const A F0 = A(p.F[0]), F1 = A(p.F[1]), F2 = A(p.F[2]);
    // rho0 + drho and j + F/2 formed in FP64, then taken to A
    const A rho = A(p.rho0 + m.s), inv_rho = A(1) / rho;
    const A ux = A(m.jx + 0.5 * p.F[0]) * inv_rho;
    const A uy = A(m.jy + 0.5 * p.F[1]) * inv_rho;
    const A uz = A(m.jz + 0.5 * p.F[2]) * inv_rho;
    A vx, vy, vz;
    sh.eq(ux, uy, uz, vx, vy, vz);
    A P0 = 0, Px = 0, Py = 0, Pz = 0;
    A Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const A wp = A(L::w[i]) * pb[i];
        P0 += wp;
        if (L::cx[i]) Px += L::cx[i] > 0 ? wp : -wp;
        if (L::cy[i]) Py += L::cy[i] > 0 ? wp : -wp;
        if (L::cz[i]) Pz += L::cz[i] > 0 ? wp : -wp;
        if (L::cx[i]) Pxx += wp;
        if (L::cy[i]) Pyy += wp;
        if (L::cz[i]) Pzz += wp;
        if (L::cx[i] * L::cy[i]) Pxy += L::cx[i] * L::cy[i] > 0 ? wp : -wp;
        if (L::cx[i] * L::cz[i]) Pxz += L::cx[i] * L::cz[i] > 0 ? wp : -wp;
        if (L::cy[i] * L::cz[i]) Pyz += L::cy[i] * L::cz[i] > 0 ? wp : -wp;
    }
    const A Pvx = Pxx * vx + Pxy * vy + Pxz * vz;
    const A Pvy = Pxy * vx + Pyy * vy + Pyz * vz;
    const A Pvz = Pxz * vx + Pyz * vy + Pzz * vz;
    const A vv = vx * vx + vy * vy + vz * vz;
    const A A_rho = P0 * (A(1) - A(1.5) * vv) + A(3) * (Px * vx + Py * vy + Pz * vz) +
                    A(4.5) * (vx * Pvx + vy * Pvy + vz * Pvz);
    const A Avx = rho * (A(3) * Px + A(9) * Pvx - A(3) * vx * P0);
    const A Avy = rho * (A(3) * Py + A(9) * Pvy - A(3) * vy * P0);
    const A Avz = rho * (A(3) * Pz + A(9) * Pvz - A(3) * vz * P0);
    const A PFx = Pxx * F0 + Pxy * F1 + Pxz * F2;
    const A PFy = Pxy * F0 + Pyy * F1 + Pyz * F2;
    const A PFz = Pxz * F0 + Pyz * F1 + Pzz * F2;
    A mAx, mAy, mAz;
    sh.om_m(om, Avx, Avy, Avz, mAx, mAy, mAz);
    const A ubx = mAx + pref * (A(9) * PFx - A(3) * F0 * P0);
    const A uby = mAy + pref * (A(9) * PFy - A(3) * F1 * P0);
    const A ubz = mAz + pref * (A(9) * PFz - A(3) * F2 * P0);
    const A rbar = om * A_rho - (ubx * ux + uby * uy + ubz * uz) * inv_rho;
    const A jbx = ubx * inv_rho, jby = uby * inv_rho, jbz = ubz * inv_rho;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        pb[k] = (A(1) - om) * pb[k] + rbar + A(L::cx[k]) * jbx + A(L::cy[k]) * jby + A(L::cz[k]) * jbz;
    sh.grad(om, Avx, Avy, Avz, ux, uy, uz, g);
}

// ---------------------------------------------------------------------------
// One reverse step t: lam_out = lambda_t from lam_in = lambda_{t+1}, with the
// forward step's moment record in `rec`; each control row of dbar += this
// step's cotangent of that row (added in FP64).
// ---------------------------------------------------------------------------
template <class L, class S, int BC, int PK>
__device__ __forceinline__ void adjoint_cell(const LamT<S>* __restrict__ lam_in, LamT<S>* __restrict__ lam_out,
                                             const LamT<S>* __restrict__ rec,
                                             const typename S::D* __restrict__ dfield, double* __restrict__ dbar,
                                             const Params& p, uint32_t x, uint32_t y, uint32_t z)
{
    using A = LamT<S>;
    const uint32_t N = p.N;
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const Moms m = recorded_moments(rec, N, cell);
    using Sh = AdjShift<PK, A>;
    const Sh sh = Sh::template load<S>(dfield, p.P, cell);  // control rows are P apart
    A pb[L::Q];
    bool solid = false;
    if (BC == BC_PERIODIC) {
        stream_adjoint_periodic<L, A>(lam_in, p.P, p, x, y, z, pb);
    } else {
        const Box b = box_of(p);
        // post-collision density and velocity of this cell at step t, from
        // the recorded moments by the balance laws (open faces only)
        auto post = [&](A& rho, A& ubx, A& uby, A& ubz) {
            rho = A(p.rho0 + m.s);
            const A inv_rho = A(1) / rho;
            const A om = A(p.omega);
            A rvx, rvy, rvz;  // omega rho u_eq = omega M (j + F/2)
            sh.om_m(om, A(m.jx + 0.5 * p.F[0]), A(m.jy + 0.5 * p.F[1]), A(m.jz + 0.5 * p.F[2]), rvx, rvy, rvz);
            ubx = ((A(1) - om) * A(m.jx) + rvx + A(p.pref * p.F[0])) * inv_rho;
            uby = ((A(1) - om) * A(m.jy) + rvy + A(p.pref * p.F[1])) * inv_rho;
            ubz = ((A(1) - om) * A(m.jz) + rvz + A(p.pref * p.F[2])) * inv_rho;
        };
        A rho_b, ubx, uby, ubz;
        if (BC == BC_PLAIN_ROW) {
            // the periodic transpose, then the row's x ends
            stream_adjoint_periodic<L, A>(lam_in, p.P, p, x, y, z, pb);
            const bool at_lo = (int)x == x_end_lo(b.lo0), at_hi = (int)x == x_end_hi(b.hi0, b.nx);
            if (at_lo | at_hi) {
                post(rho_b, ubx, uby, ubz);
                stream_adjoint_x_ends<L, A>(lam_in, p.P, p, b, at_lo, at_hi, cell, rho_b, ubx, uby, ubz, pb);
            }
        } else {
            post(rho_b, ubx, uby, ubz);
            stream_adjoint_general<L, A>(lam_in, p.P, p, (int)x, (int)y, (int)z, rho_b, ubx, uby, ubz, pb);
        }
        solid = in_wall_layer(b, (int)x, (int)y, (int)z);
    }
    A g[Sh::rows];
    collide_adjoint<L, A>(m, sh, p, pb, g);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) st(lam_out + (size_t)k * p.P, cell, sel(solid, A(0), pb[k]));
#pragma unroll
    for (int r = 0; r < Sh::rows; ++r) {
        // FP64 gradient rows can pass 4 GiB: 64-bit indexing
        double* const at = dbar + (size_t)r * N + cell;
        *at = *at + double(sel(solid, A(0), g[r]));
    }
}

template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(256) void adjoint_kernel(const LamT<S>* __restrict__ lam_in,
                                                       LamT<S>* __restrict__ lam_out,
                                                       const LamT<S>* __restrict__ rec,
                                                       const typename S::D* __restrict__ dfield,
                                                       double* __restrict__ dbar, Params p)
{
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    if (BC != BC_GENERAL) {
        adjoint_cell<L, S, BC, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, blockIdx.y, blockIdx.z);
        return;
    }
    // with walls or open faces the rows are taken in row_of order (the rows
    // that are not plain first); plain rows take the periodic transpose and
    // their x ends, the others the general rule; the choice is uniform per
    // block and each path keeps its own collision and stores
    int y, z;
    row_of((int)(blockIdx.y + gridDim.y * blockIdx.z), p.ny, p.nz, p.bc_lo[1], p.bc_hi[1], p.bc_lo[2], p.bc_hi[2],
           y, z);
    if (plain_row(y, z, p.ny, p.nz, p.bc_lo[1], p.bc_hi[1], p.bc_lo[2], p.bc_hi[2]))
        adjoint_cell<L, S, BC_PLAIN_ROW, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, (uint32_t)y, (uint32_t)z);
    else
        adjoint_cell<L, S, BC, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, (uint32_t)y, (uint32_t)z);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <class L, class S>
static hipError_t seed_dispatch_bc(int bcmode, const Params& p, const void* src, const double* drho_bar,
                                   const double* u_bar, void* lam, int bx, hipStream_t s)
{
    const Launch l = cell_launch(p, bx < 256 ? bx : 256);
    auto* a = static_cast<const typename S::T*>(src);
    if (bcmode == BC_PERIODIC)
        hipLaunchKernelGGL((adjoint_seed_kernel<L, S, BC_PERIODIC>), l.grid, l.block, 0, s, a, drho_bar,
                           u_bar, static_cast<LamT<S>*>(lam), p);
    else
        hipLaunchKernelGGL((adjoint_seed_kernel<L, S, BC_GENERAL>), l.grid, l.block, 0, s, a, drho_bar,
                           u_bar, static_cast<LamT<S>*>(lam), p);
    return hipGetLastError();
}

template <class L, class S, int PK>
static hipError_t adjoint_dispatch_bc(int bcmode, const Params& p, const void* lam_in, void* lam_out,
                                      const void* rec_v, const void* dfield, double* dbar, int bx, hipStream_t s)
{
    auto* rec = static_cast<const LamT<S>*>(rec_v);
    const Launch l = cell_launch(p, bx < 256 ? bx : 256);
    auto* d = static_cast<const typename S::D*>(dfield);
    auto* li = static_cast<const LamT<S>*>(lam_in);
    auto* lo = static_cast<LamT<S>*>(lam_out);
    if (bcmode == BC_PERIODIC)
        hipLaunchKernelGGL((adjoint_kernel<L, S, BC_PERIODIC, PK>), l.grid, l.block, 0, s, li, lo, rec, d, dbar, p);
    else
        hipLaunchKernelGGL((adjoint_kernel<L, S, BC_GENERAL, PK>), l.grid, l.block, 0, s, li, lo, rec, d, dbar, p);
    return hipGetLastError();
}

template <class L>
static hipError_t seed_dispatch_store(int storage, int bcmode, const Params& p, const void* src,
                                      const double* drho_bar, const double* u_bar, void* lam, int bx,
                                      hipStream_t s)
{
    switch (storage) {
    case StoreF64::code: return seed_dispatch_bc<L, StoreF64>(bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    case StoreF32::code: return seed_dispatch_bc<L, StoreF32>(bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    case StoreF16S::code: return seed_dispatch_bc<L, StoreF16S>(bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    case StoreBF16S::code: return seed_dispatch_bc<L, StoreBF16S>(bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    default: return hipErrorInvalidValue;
    }
}

template <class L, int PK>
static hipError_t adjoint_dispatch_store(int storage, int bcmode, const Params& p, const void* lam_in,
                                         void* lam_out, const void* rec, const void* dfield, double* dbar, int bx,
                                         hipStream_t s)
{
    switch (storage) {
    case StoreF64::code: return adjoint_dispatch_bc<L, StoreF64, PK>(bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    case StoreF32::code: return adjoint_dispatch_bc<L, StoreF32, PK>(bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    case StoreF16S::code:
        return adjoint_dispatch_bc<L, StoreF16S, PK>(bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    case StoreBF16S::code:
        return adjoint_dispatch_bc<L, StoreBF16S, PK>(bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_seed(int q, int storage, int bcmode, const Params& p, const void* src,
                               const double* drho_bar, const double* u_bar, void* lam, int bx,
                               hipStream_t s)
{
    if (q == 9) return seed_dispatch_store<D2Q9>(storage, bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    if (q == 19) return seed_dispatch_store<D3Q19>(storage, bcmode, p, src, drho_bar, u_bar, lam, bx, s);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int q, int storage, int bcmode, int pk, const Params& p, const void* lam_in,
                          void* lam_out, const void* dfield, double* dbar, int bx, hipStream_t s,
                          const void* moment_record)
{
    const void* rec = moment_record;
    if (!rec) return hipErrorInvalidValue;
    if (q == 9 && pk == PK_SCALAR)
        return adjoint_dispatch_store<D2Q9, PK_SCALAR>(storage, bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    if (q == 19 && pk == PK_SCALAR)
        return adjoint_dispatch_store<D3Q19, PK_SCALAR>(storage, bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    if (q == 19 && pk == PK_TENSOR)
        return adjoint_dispatch_store<D3Q19, PK_TENSOR>(storage, bcmode, p, lam_in, lam_out, rec, dfield, dbar, bx, s);
    return hipErrorInvalidValue;
}

}  // namespace hlbm
