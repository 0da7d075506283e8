// Discrete adjoint of the sweep (reverse mode) for gradients of an objective
// of the moments with respect to the porosity control: d = 1 - varpi
// (Sec. 3.2), or the six rows xx, yy, zz, xy, xz, yz of a symmetric tensor D
// (u_eq = (I - D) u; an off-diagonal row is one variable at two places).
//
// One forward step is y_t = S(x_{t-1}) (pull streaming) followed by
// x_t = C(y_t, d) (the homogenized BGK collision of Sec. 3.2, cell-local), and
// the objective observes the moments M(S(x_T)).  The reverse sweep carries the
// adjoint of the pre-collision populations, lambda_t = dJ/dy_t, in FP64:
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
// the forward state's rows, FP64 for the FP64 form and FP32 for the others; all adjoint
// arithmetic is FP64 and dJ/dd is one FP64 value per cell and control row,
// accumulated.  Blocks
// hold at most 256 threads (the FP64 adjoint needs more registers than a
// 1024-thread block leaves per thread); the launchers clamp the block width.
#include <type_traits>

#include "cell.hpp"

namespace hlbm {

// Element type of the adjoint populations for storage policy S.
template <class S>
using LamT = typename std::conditional<std::is_same<S, StoreF64>::value, double, float>::type;

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
template <class L, class LT>
__device__ __forceinline__ void stream_adjoint_periodic(const LT* __restrict__ lam, uint32_t P,
                                                        const Params& p, uint32_t x, uint32_t y,
                                                        uint32_t z, double (&pb)[L::Q])
{
    const uint32_t nx = p.nx, ny = p.ny, nz = p.nz;
    // x + c for c = -1, 0, +1 (index c + 1), wrapped
    const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x + 1 == nx ? 0u : x + 1};
    const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0u : y + 1};
    const uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z + 1 == nz ? 0u : z + 1};
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const uint32_t off = xs[L::cx[k] + 1] + nx * (ys[L::cy[k] + 1] + ny * zs[L::cz[k] + 1]);
        pb[k] = (double)ld(lam + (size_t)k * P, off);
    }
}

// Walls and open faces.  `rho_b`, (ubx, uby, ubz) are this cell's
// post-collision density and velocity j_b/rho_b at the forward step whose
// open-face equilibria are being differentiated.
template <class L, class LT>
__device__ __forceinline__ void stream_adjoint_general(const LT* __restrict__ lam, uint32_t P,
                                                       const Params& p, int x, int y, int z,
                                                       double rho_b, double ubx, double uby,
                                                       double ubz, double (&pb)[L::Q])
{
    const Box b = box_of(p);
    const uint32_t cell = (uint32_t)x + (uint32_t)b.nx * ((uint32_t)y + (uint32_t)b.ny * (uint32_t)z);
    const bool px = b.lo0 == 0, py = b.lo1 == 0, pz = b.lo2 == 0;
    const double uix = p.inlet_u[0], uiy = p.inlet_u[1], uiz = p.inlet_u[2];
    const double uin2 = uix * uix + uiy * uiy + uiz * uiz;
    const double rout = p.outlet_rho;
    double a_in = 0.0, bvx = 0.0, bvy = 0.0, bvz = 0.0;
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
        const double v = (double)ld(lam + (size_t)row * P, off);
        const bool open = outside & !wall;
        pb[k] = sel(open, 0.0, v);
        // open face: v is the adjoint of this cell's pre-collision population
        // i = opp(k), which the forward step took from an equilibrium
        const int kx = sel(sx < 0, b.lo0, b.hi0);
        const int ky = sel(sy < 0, b.lo1, b.hi1);
        const int kz = sel(sz < 0, b.lo2, b.hi2);
        const int kind = sel(out_x, kx, sel(out_y, ky, kz));
        const bool inlet = kind == 2;
        const int i = opposite(k);
        const double w = L::w[i];
        const double cix = L::cx[i], ciy = L::cy[i], ciz = L::cz[i];
        const double cin = cix * uix + ciy * uiy + ciz * uiz;
        // inlet f^eq(rho_b, u_in): d/d rho_b
        const double d_in = w * (1.0 + 3.0 * cin + 4.5 * cin * cin - 1.5 * uin2);
        a_in += sel(open & inlet, v * d_in, 0.0);
        // outlet f^eq(rho_out, u_b): d/d u_b
        const double cub = cix * ubx + ciy * uby + ciz * ubz;
        const double wv = sel(open & !inlet, v * w * rout, 0.0);
        bvx += wv * (3.0 * cix + 9.0 * cub * cix - 3.0 * ubx);
        bvy += wv * (3.0 * ciy + 9.0 * cub * ciy - 3.0 * uby);
        bvz += wv * (3.0 * ciz + 9.0 * cub * ciz - 3.0 * ubz);
    }
    // rho_b depends on every own population with weight 1, u_b = j_b/rho_b
    const double inv_b = 1.0 / rho_b;
    const double common = a_in - (bvx * ubx + bvy * uby + bvz * ubz) * inv_b;
    const double gx = bvx * inv_b, gy = bvy * inv_b, gz = bvz * inv_b;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        pb[k] += common + double(L::cx[k]) * gx + double(L::cy[k]) * gy + double(L::cz[k]) * gz;
}

// ---------------------------------------------------------------------------
// The control in the adjoint's FP64: u_eq = M u with M = (1 - d) I (scalar) or
// M = I - D (tensor; symmetric, so M^T = M).
//   om_m(om, a) = omega M a
//   grad(om, Av, u, g): g_r = omega Av . (dM/dtheta_r) u, the cotangent of
//   control row r, with dM/dd = -I for the scalar d, -e_a e_a^T for a
//   diagonal row and -(e_a e_b^T + e_b e_a^T) for an off-diagonal row (a, b).
// ---------------------------------------------------------------------------
struct AdjScalar {
    static constexpr int rows = 1;
    double d;
    template <class S>
    __device__ __forceinline__ static AdjScalar load(const typename S::D* __restrict__ f, uint32_t, uint32_t cell)
    {
        return AdjScalar{(double)S::load_d(ld(f, cell))};
    }
    __device__ __forceinline__ void eq(double ux, double uy, double uz, double& vx, double& vy, double& vz) const
    {
        const double sh = 1.0 - d;
        vx = sh * ux;
        vy = sh * uy;
        vz = sh * uz;
    }
    __device__ __forceinline__ void om_m(double om, double ax, double ay, double az, double& bx, double& by,
                                         double& bz) const
    {
        const double s = om * (1.0 - d);
        bx = s * ax;
        by = s * ay;
        bz = s * az;
    }
    __device__ __forceinline__ void grad(double om, double Avx, double Avy, double Avz, double ux, double uy,
                                         double uz, double (&g)[1]) const
    {
        g[0] = -om * (Avx * ux + Avy * uy + Avz * uz);
    }
};

struct AdjTensor {
    static constexpr int rows = 6;
    double xx, yy, zz, xy, xz, yz;
    template <class S>
    __device__ __forceinline__ static AdjTensor load(const typename S::D* __restrict__ f, uint32_t pitch,
                                                     uint32_t cell)
    {
        return AdjTensor{(double)S::load_d(ld(f, cell)),
                         (double)S::load_d(ld(f + (size_t)pitch, cell)),
                         (double)S::load_d(ld(f + 2 * (size_t)pitch, cell)),
                         (double)S::load_d(ld(f + 3 * (size_t)pitch, cell)),
                         (double)S::load_d(ld(f + 4 * (size_t)pitch, cell)),
                         (double)S::load_d(ld(f + 5 * (size_t)pitch, cell))};
    }
    __device__ __forceinline__ void eq(double ux, double uy, double uz, double& vx, double& vy, double& vz) const
    {
        vx = ux - (xx * ux + xy * uy + xz * uz);
        vy = uy - (xy * ux + yy * uy + yz * uz);
        vz = uz - (xz * ux + yz * uy + zz * uz);
    }
    __device__ __forceinline__ void om_m(double om, double ax, double ay, double az, double& bx, double& by,
                                         double& bz) const
    {
        double mx, my, mz;
        eq(ax, ay, az, mx, my, mz);
        bx = om * mx;
        by = om * my;
        bz = om * mz;
    }
    __device__ __forceinline__ void grad(double om, double Avx, double Avy, double Avz, double ux, double uy,
                                         double uz, double (&g)[6]) const
    {
        g[0] = -om * (Avx * ux);
        g[1] = -om * (Avy * uy);
        g[2] = -om * (Avz * uz);
        g[3] = -om * (Avx * uy + Avy * ux);
        g[4] = -om * (Avx * uz + Avz * ux);
        g[5] = -om * (Avy * uz + Avz * uy);
    }
};

template <int PK>
using AdjShift = typename std::conditional<PK == PK_TENSOR, AdjTensor, AdjScalar>::type;

// ---------------------------------------------------------------------------
// C^T of one fluid cell.  In: the FP64 moments of y, the control, and pb =
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
template <class L, class Sh>
__device__ __forceinline__ void collide_adjoint(const Moms& m, const Sh& sh, const Params& p,
                                                double (&pb)[L::Q], double (&g)[Sh::rows])
{
    const double om = p.omega, pref = p.pref;
    const double F0 = p.F[0], F1 = p.F[1], F2 = p.F[2];
    const double rho = p.rho0 + m.s, inv_rho = 1.0 / rho;
    const double ux = (m.jx + 0.5 * F0) * inv_rho;
    const double uy = (m.jy + 0.5 * F1) * inv_rho;
    const double uz = (m.jz + 0.5 * F2) * inv_rho;
    double vx, vy, vz;
    sh.eq(ux, uy, uz, vx, vy, vz);
    double P0 = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
    double Pxx = 0.0, Pyy = 0.0, Pzz = 0.0, Pxy = 0.0, Pxz = 0.0, Pyz = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double wp = L::w[i] * pb[i];
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
    const double Pvx = Pxx * vx + Pxy * vy + Pxz * vz;
    const double Pvy = Pxy * vx + Pyy * vy + Pyz * vz;
    const double Pvz = Pxz * vx + Pyz * vy + Pzz * vz;
    const double vv = vx * vx + vy * vy + vz * vz;
    const double A_rho = P0 * (1.0 - 1.5 * vv) + 3.0 * (Px * vx + Py * vy + Pz * vz) +
                         4.5 * (vx * Pvx + vy * Pvy + vz * Pvz);
    const double Avx = rho * (3.0 * Px + 9.0 * Pvx - 3.0 * vx * P0);
    const double Avy = rho * (3.0 * Py + 9.0 * Pvy - 3.0 * vy * P0);
    const double Avz = rho * (3.0 * Pz + 9.0 * Pvz - 3.0 * vz * P0);
    const double PFx = Pxx * F0 + Pxy * F1 + Pxz * F2;
    const double PFy = Pxy * F0 + Pyy * F1 + Pyz * F2;
    const double PFz = Pxz * F0 + Pyz * F1 + Pzz * F2;
    double mAx, mAy, mAz;
    sh.om_m(om, Avx, Avy, Avz, mAx, mAy, mAz);
    const double ubx = mAx + pref * (9.0 * PFx - 3.0 * F0 * P0);
    const double uby = mAy + pref * (9.0 * PFy - 3.0 * F1 * P0);
    const double ubz = mAz + pref * (9.0 * PFz - 3.0 * F2 * P0);
    const double rbar = om * A_rho - (ubx * ux + uby * uy + ubz * uz) * inv_rho;
    const double jbx = ubx * inv_rho, jby = uby * inv_rho, jbz = ubz * inv_rho;
#pragma unroll
    for (int k = 0; k < L::Q; ++k)
        pb[k] = (1.0 - om) * pb[k] + rbar + double(L::cx[k]) * jbx + double(L::cy[k]) * jby +
                double(L::cz[k]) * jbz;
    sh.grad(om, Avx, Avy, Avz, ux, uy, uz, g);
}

// ---------------------------------------------------------------------------
// One reverse step t: lam_out = lambda_t from lam_in = lambda_{t+1}, with the
// forward step's moment record in `rec`; each control row of dbar += this
// step's cotangent of that row.
// ---------------------------------------------------------------------------
template <class L, class S, int BC, int PK>
__device__ __forceinline__ void adjoint_cell(const LamT<S>* __restrict__ lam_in, LamT<S>* __restrict__ lam_out,
                                             const double* __restrict__ rec,
                                             const typename S::D* __restrict__ dfield, double* __restrict__ dbar,
                                             const Params& p, uint32_t x, uint32_t y, uint32_t z)
{
    const uint32_t N = p.N;
    const uint32_t cell = x + (uint32_t)p.nx * (y + (uint32_t)p.ny * z);
    const Moms m = recorded_moments(rec, N, cell);
    using Sh = AdjShift<PK>;
    const Sh sh = Sh::template load<S>(dfield, p.P, cell);  // control rows are P apart
    double pb[L::Q];
    bool solid = false;
    if (BC == BC_PERIODIC) {
        stream_adjoint_periodic<L, LamT<S>>(lam_in, p.P, p, x, y, z, pb);
    } else {
        // post-collision moments of this cell at step t (balance laws)
        const double rho = p.rho0 + m.s, inv_rho = 1.0 / rho;
        const double om = p.omega;
        double rvx, rvy, rvz;  // omega rho u_eq = omega M (j + F/2)
        sh.om_m(om, m.jx + 0.5 * p.F[0], m.jy + 0.5 * p.F[1], m.jz + 0.5 * p.F[2], rvx, rvy, rvz);
        const double jbx = (1.0 - om) * m.jx + rvx + p.pref * p.F[0];
        const double jby = (1.0 - om) * m.jy + rvy + p.pref * p.F[1];
        const double jbz = (1.0 - om) * m.jz + rvz + p.pref * p.F[2];
        stream_adjoint_general<L, LamT<S>>(lam_in, p.P, p, (int)x, (int)y, (int)z, rho, jbx * inv_rho,
                                  jby * inv_rho, jbz * inv_rho, pb);
        solid = in_wall_layer(box_of(p), (int)x, (int)y, (int)z);
    }
    double g[Sh::rows];
    collide_adjoint<L>(m, sh, p, pb, g);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) st(lam_out + (size_t)k * p.P, cell, LamT<S>(sel(solid, 0.0, pb[k])));
#pragma unroll
    for (int r = 0; r < Sh::rows; ++r) {
        // FP64 gradient rows can pass 4 GiB: 64-bit indexing
        double* const at = dbar + (size_t)r * N + cell;
        *at = *at + sel(solid, 0.0, g[r]);
    }
}

template <class L, class S, int BC, int PK>
__global__ __launch_bounds__(256) void adjoint_kernel(const LamT<S>* __restrict__ lam_in,
                                                       LamT<S>* __restrict__ lam_out,
                                                       const double* __restrict__ rec,
                                                       const typename S::D* __restrict__ dfield,
                                                       double* __restrict__ dbar, Params p)
{
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)p.nx) return;
    adjoint_cell<L, S, BC, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, blockIdx.y, blockIdx.z);
}

// Interior and shell of a box with walls or open faces (see Split), in one
// launch: in the interior the periodic forms of the gather and of its
// transpose load what the general rule would; the shell takes the general
// rule.  The choice is uniform per block.  The shell's blocks come first:
// they are the slow ones, and blocks start in index order, so the interior
// blocks fill in behind them instead of leaving them as the tail.
template <class L, class S, int PK>
__global__ __launch_bounds__(256) void adjoint_split_kernel(const LamT<S>* __restrict__ lam_in,
                                                             LamT<S>* __restrict__ lam_out,
                                                             const double* __restrict__ rec,
                                                             const typename S::D* __restrict__ dfield,
                                                             double* __restrict__ dbar, Params p, Split sp)
{
    const uint32_t b = blockIdx.x;
    if (b < sp.blocks_shell) {
        const uint32_t k = b * blockDim.x + threadIdx.x;
        if (k >= sp.n_shell) return;
        uint32_t x, y, z;
        shell_cell(sp, (uint32_t)p.nx, (uint32_t)p.ny, k, x, y, z);
        adjoint_cell<L, S, BC_GENERAL, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, y, z);
    } else {
        const uint32_t bi = b - sp.blocks_shell;
        const uint32_t row = bi / sp.gx, bxi = bi - row * sp.gx;
        const uint32_t iy = sp.hi[1] - sp.lo[1];
        const uint32_t zz = row / iy, yy = row - zz * iy;
        const uint32_t x = sp.lo[0] + bxi * blockDim.x + threadIdx.x;
        if (x >= sp.hi[0]) return;
        adjoint_cell<L, S, BC_PERIODIC, PK>(lam_in, lam_out, rec, dfield, dbar, p, x, sp.lo[1] + yy, sp.lo[2] + zz);
    }
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
                                      const double* rec, const void* dfield, double* dbar, int bx, hipStream_t s)
{
    const Launch l = cell_launch(p, bx < 256 ? bx : 256);
    auto* d = static_cast<const typename S::D*>(dfield);
    auto* li = static_cast<const LamT<S>*>(lam_in);
    auto* lo = static_cast<LamT<S>*>(lam_out);
    if (bcmode == BC_PERIODIC) {
        hipLaunchKernelGGL((adjoint_kernel<L, S, BC_PERIODIC, PK>), l.grid, l.block, 0, s, li, lo, rec, d, dbar, p);
        return hipGetLastError();
    }
    const Split sp = split_of(p, (int)l.block.x);
    if (!sp.interior()) {
        hipLaunchKernelGGL((adjoint_kernel<L, S, BC_GENERAL, PK>), l.grid, l.block, 0, s, li, lo, rec, d, dbar, p);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((adjoint_split_kernel<L, S, PK>), dim3(sp.blocks_in + sp.blocks_shell), l.block, 0, s, li, lo,
                       rec, d, dbar, p, sp);
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
                                         void* lam_out, const double* rec, const void* dfield, double* dbar, int bx,
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
                          const double* moment_record)
{
    const double* rec = moment_record;
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
