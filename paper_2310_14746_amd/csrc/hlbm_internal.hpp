// Internal declarations shared by the kernels (sweep.hip) and the C-ABI host
// code (api.hip).  Not installed; the public interface is include/hlbm.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hlbm {

// Per-launch constants of the sweep, passed by value in the kernel arguments.
struct Params {
    int nx, ny, nz;
    uint32_t N;          // cells = nx*ny*nz (< 2^32)
    uint32_t P;          // elements from one population row to the next (>= N, see row_pitch)
    double omega;        // 1/tau
    double pref;         // 1 - 1/(2 tau), Guo source prefactor
    double F[3];         // body-force density
    double rho0;         // reference density of the shifted populations
    double scale;        // 16-bit storage scale s (power of two), else 1
    double inv_scale;    // 1/s
    int bc_lo[3];        // face kinds (HLBM_PERIODIC, HLBM_WALL, ...)
    int bc_hi[3];
    double inlet_u[3];
    double outlet_rho;
    const uint32_t* linkmask;  // BC_MASKED: per cell, bit i = source of direction i is solid,
                               // bit 31 = the cell itself is solid (else unused)
};

// BC_MASKED: periodic box with resolved solid cells (bounce-back links).
// BC_AA_EVEN / BC_AA_ODD: the two steps of the in-place (AA) pattern in a
// periodic box.  Even step: the cell reads its own slots, which hold its
// pulled pre-collision populations, and writes post-collision population i to
// its own slot opp(i).  Odd step: it reads population i from slot opp(i) of
// x - c_i and writes post-collision population i to slot i of x + c_i.  Each
// slot is read and written by one thread per step, so one buffer suffices,
// and the arithmetic is that of the A/B pull bit for bit.
// BC_AA_EVEN_W / BC_AA_ODD_W: the same steps with wall faces (periodic or
// wall on every axis).  In the odd step a population whose source is solid is
// read from the cell's own slot i (halfway bounce-back: the even step left
// the cell's post-collision population opp(i) there), and a post-collision
// population whose target is solid is written to the cell's own slot opp(i)
// (where the even step expects the bounced population).  Those slots belong
// to the solid neighbour, which touches only its own slots, so the pattern
// stays free of races.  Solid cells store zeros, as in the A/B sweep.
enum BcMode {
    BC_PERIODIC = 0,
    BC_GENERAL = 1,
    BC_MASKED = 2,
    BC_AA_EVEN = 3,
    BC_AA_ODD = 4,
    BC_AA_EVEN_W = 5,
    BC_AA_ODD_W = 6,
    // device-side only: a plain row (see plain_row) inside the BC_GENERAL
    // kernels, which choose it per row
    BC_PLAIN_ROW = 7
};
constexpr uint32_t LINK_SOLID_SELF = 1u << 31;

// Population rows may run `pad_bytes` past their N cells (hlbm_config::
// row_pad_bytes, a multiple of 256).  A box whose row is a large power of two
// (512^3 FP32: 512 MiB) otherwise starts every one of the 19 rows at the same
// offset modulo every power of two up to the row size, and the 19 concurrent
// read streams of a wave and the 19 write streams fall on the same HBM
// channels together; shifting row i by i * pad spreads them.  Snapshots
// (hlbm_get_state / hlbm_set_state) keep the dense layout of N per row.
constexpr int ROW_PAD_MAX = 1 << 24;
inline uint32_t row_pitch(uint32_t n, size_t elem, int pad_bytes) { return n + (uint32_t)(pad_bytes / elem); }
// Porosity control kinds: one value d per cell, or a symmetric 3x3 D (6 rows).
enum PorosityKind { PK_SCALAR = 0, PK_TENSOR = 1 };

// Boxes with walls or open faces: which pulls need the boundary rules.  Face
// kinds: 0 periodic, 1 wall, 2 inlet, 3 outlet.  Along an axis, the cells
// whose pulls cross a face are its depth layers: a wall face's solid layer and
// the layer that bounces back against it (2), an open face's own layer (1),
// none on a periodic axis.
__host__ __device__ inline int face_depth(int kind) { return kind == 0 ? 0 : (kind == 1 ? 2 : 1); }

// A plain row (y, z): no pull of any of its cells crosses a y or z face, so
// the periodic gather (and its transpose) loads what the boundary rules would
// everywhere but at the row's x ends.  Bitwise operators: no branches.
__host__ __device__ inline bool plain_row(int y, int z, int ny, int nz, int lo1, int hi1, int lo2, int hi2)
{
    return (int(y >= face_depth(lo1)) & int(y < ny - face_depth(hi1)) & int(z >= face_depth(lo2)) &
            int(z < nz - face_depth(hi2))) != 0;
}

// Row order of the kernels with walls or open faces: row r (r = blockIdx.y +
// ny blockIdx.z) -> (y, z), the rows that are not plain first (they take the
// slower general rule, and blocks start in index order, so the plain rows
// fill in behind them instead of leaving them as the tail), then the plain
// rows, each part in z-major order.  A bijection of [0, ny nz); scalar
// arithmetic with selects, once per block.
__host__ __device__ inline void row_of(int r, int ny, int nz, int lo1, int hi1, int lo2, int hi2, int& y, int& z)
{
    const int ylo = face_depth(lo1), zlo = face_depth(lo2);
    const int yhi = ny - face_depth(hi1) > ylo ? ny - face_depth(hi1) : ylo;
    const int zhi = nz - face_depth(hi2) > zlo ? nz - face_depth(hi2) : zlo;
    const int iy = yhi - ylo, iz = zhi - zlo;
    const int general = ny * nz - iy * iz;
    const int below = zlo * ny, mid = iz * (ny - iy);
    // every candidate, then selects (no branches; a discarded candidate's
    // divisor is never zero)
    const int q4 = r - general, d4 = iy > 0 ? iy : 1;  // plain rows
    const int z4 = zlo + q4 / d4, y4 = ylo + q4 % d4;
    const int z1 = r / ny, y1 = r % ny;  // planes below the plain z range
    const int q2 = r - below, wy = ny - iy > 0 ? ny - iy : 1;  // plain z range, y outside
    const int z2 = zlo + q2 / wy, yy2 = q2 % wy;
    const int y2 = yy2 < ylo ? yy2 : yhi + (yy2 - ylo);
    const int q3 = r - below - mid;  // planes above
    const int z3 = zhi + q3 / ny, y3 = q3 % ny;
    const bool plain = r >= general, lower = r < below, middle = r < below + mid;
    z = plain ? z4 : (lower ? z1 : (middle ? z2 : z3));
    y = plain ? y4 : (lower ? y1 : (middle ? y2 : y3));
}

// The x end cells of a plain row whose pulls cross an x face: at the lo face
// x = 0 beside an open face and x = 1 beside a wall (whose solid layer x = 0
// pulls nothing that is kept), and likewise at the hi face; -1 on a periodic
// axis.  Directions with c_x = +1 cross the lo face there, c_x = -1 the hi
// face (the adjoint's transposed pulls: the opposite directions).
__host__ __device__ inline int x_end_lo(int lo0) { return lo0 == 0 ? -1 : face_depth(lo0) - 1; }
__host__ __device__ inline int x_end_hi(int hi0, int nx) { return hi0 == 0 ? -1 : nx - face_depth(hi0); }

// Launch geometry shared by every per-cell kernel: blocks of `bx` threads
// along x, grid (ceil(nx/bx), ny, nz).
struct Launch {
    dim3 grid, block;
    uint32_t nblocks;
};
Launch cell_launch(const Params& p, int bx, int cells_per_thread = 1);

// Kernel launchers (sweep.hip).  All return the launch status.
// One sweep.  With diag_partials != NULL the diagnostic variant also writes
// FP64 block partials of the totals (one 4-double record per block).
// With moment_record != NULL (A/B, periodic or general faces, no diagnostics)
// the sweep also writes each cell's pre-collision moments s, jx, jy, jz (the
// reverse sweep's linearization point) there as four rows of N values of
// adjoint_elem_bytes(storage) bytes (the FP64 sums, rounded to FP32 for the
// forms other than FP64).
hipError_t launch_sweep(int q, int storage, int bcmode, int pk, const Params& p, const void* src,
                        void* dst, const void* dfield, int bx, hipStream_t s,
                        double* diag_partials = nullptr, void* moment_record = nullptr);
hipError_t launch_moments(int q, int storage, int bcmode, const Params& p, const void* src,
                          void* drho, void* u, int out_f64, double* partials, int bx,
                          hipStream_t s);
// Reverse sweep (adjoint.hip): seed from the moments' cotangents, then one
// launch per reverse step.  Adjoint populations are rows of N values of
// adjoint_elem_bytes(storage) bytes (FP64 for the FP64 form, FP32 otherwise).
inline size_t adjoint_elem_bytes(int storage) { return storage == 0 ? 8 : 4; }
hipError_t launch_adjoint_seed(int q, int storage, int bcmode, const Params& p, const void* src,
                               const double* drho_bar, const double* u_bar, void* lam, int bx,
                               hipStream_t s);
// dbar holds one row of N values per row of the control (1 scalar, 6 tensor).
// The forward step's moments come from its moment record, as the recording
// sweep of launch_sweep wrote it.
hipError_t launch_adjoint(int q, int storage, int bcmode, int pk, const Params& p, const void* lam_in,
                          void* lam_out, const void* dfield, double* dbar, int bx, hipStream_t s,
                          const void* moment_record);
// Fixed-order two-pass sum of `nblocks` partials of 4 doubles into out[4];
// `stage` holds 4*REDUCE_STAGE doubles.
constexpr uint32_t REDUCE_STAGE = 256;
// Link mask of a solid mask (uint8 per cell, nonzero = solid), periodic box.
hipError_t launch_linkmask(int q, const Params& p, const unsigned char* mask, uint32_t* linkmask,
                           hipStream_t s);
// AA-pattern state export (periodic box): the post-collision populations in
// A/B layout from the AA buffer (odd_ready: the buffer holds them in opposite
// slots; else it holds the pulled populations in natural slots).  out must not
// overlap buf.
hipError_t launch_aa_export(int q, int storage, const Params& p, const void* buf, void* out, int odd_ready,
                            hipStream_t s);
hipError_t launch_reduce4(const double* partials, uint32_t nblocks, double* stage, double* out,
                          hipStream_t s);
// Convert and validate the porosity; *flag (device) ends nonzero if any value
// is NaN or outside [0, 1].
// A tensor control's six rows are written `pitch` elements apart.
hipError_t launch_porosity_convert(int in_dtype, const void* in, int storage, int pk, void* out,
                                   uint32_t n, uint32_t pitch, int* flag, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched periodic boxes
// ---------------------------------------------------------------------------
// Schedule of the batched kernels: a tile is `tile` consecutive cells of one
// item and one block of `tile` threads; the persistent kernel keeps
// `blocks_per_cu` blocks resident per CU and draws `chunk` tiles at a time.
constexpr int TILE_DEFAULT = 256;
constexpr int TILE_MAX = 512;   // FP64 needs more than the 128 VGPRs a 1024-thread block leaves
constexpr int CHUNK_DEFAULT = 2;
constexpr int CHUNK_MAX = 64;
// default resident threads per CU of the persistent kernel (blocks_per_cu =
// this / tile, at least 1): a few waves per SIMD, so that the grid barrier
// has few participants
constexpr int BATCH_THREADS_PER_CU_DEFAULT = 512;

// One item of a batch, as read by the kernels.
struct BatchItem {
    uint32_t base;    // first cell of the item in the packed arrays
    uint32_t cells;   // nx*ny*nz
    uint32_t tile0;   // first tile of the item
    uint32_t nx, ny, nz;
    uint32_t mx, my;  // ceil(2^32/nx), ceil(2^32/ny): quotients by multiply-high
    double omega, pref;
    double F[3];
};

// Everything a batched launch needs besides the population buffers.
struct BatchLaunch {
    const BatchItem* items;     // device, n_items
    const uint32_t* tile_item;  // device, ntiles
    const uint32_t* linkmask;   // device, packed cells: solid links of items with obstacles, or null
    uint32_t n_items, ntiles;
    uint32_t Ntot;              // population row stride: packed cells plus the row pad
    double rho0, scale;
    unsigned long long* sync;   // device: [0] barrier arrivals, [1] work chunks taken
    int* err;                   // device error flag
    unsigned spin_limit;
    int grid;                   // resident blocks of the persistent kernel
    uint32_t tile;              // cells per tile = threads per block
    uint32_t chunk;             // tiles per draw of the persistent kernel
};

hipError_t launch_batch_persistent(int storage, const BatchLaunch& b, void* buf_a, void* buf_b,
                                   const void* dfield, int nsteps, int start_in_b, hipStream_t s);
hipError_t launch_batch_step(int storage, const BatchLaunch& b, const void* src, void* dst,
                             const void* dfield, hipStream_t s);
hipError_t launch_batch_moments(int storage, const BatchLaunch& b, const void* src, double* partials,
                                int sel_item, double* drho, double* u, double* totals, hipStream_t s);
hipError_t batch_occupancy(int storage, int tile, int* blocks_per_cu);
hipError_t build_batch_graph(int storage, const BatchLaunch& b, void* buf_a, void* buf_b,
                             const void* dfield, int nsteps, int start_in_b, bool persistent,
                             hipGraphExec_t* out);

}  // namespace hlbm
