// C-ABI of the HLBM sweep (declarations and contract in include/hlbm.h).
//
// Host-side validation, memory ownership, buffer swapping and error mapping.
// Every kernel launch is preceded by checks that the buffers hold the cells and
// populations the launch geometry addresses.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "hlbm.h"
#include "hlbm_internal.hpp"
#include "lattice.hpp"

using hlbm::Params;

// Polls of the persistent batch kernel's grid barrier before it gives up
// (each poll sleeps about 0.1 us): far beyond any step of the workloads here.
constexpr unsigned kBarrierPollsDefault = 1u << 20;

// Static device scratch of hlbm_moments_noalloc: the moments kernel's FP64
// block partials (4 per block, at most kScratchBlocks blocks) followed by the
// first-pass results of the two-pass reduction (4 * REDUCE_STAGE).  Every GPU
// the library runs on holds its own copy (16 MiB) until the process ends.
// Host code never passes `scratch` itself to a kernel (in host code the name
// is a stand-in, not a device address): it uses the per-device address that
// hipGetSymbolAddress returns, below.
constexpr uint32_t kScratchBlocks = 1u << 19;
constexpr size_t kScratchDoubles = 4 * ((size_t)kScratchBlocks + hlbm::REDUCE_STAGE);
static __device__ __align__(256) double scratch[kScratchDoubles];

struct hlbm_ctx {
    hlbm_config cfg;
    Params p;
    int q;
    int bcmode;
    int bx;
    size_t elem;       // bytes per stored population value
    size_t delem;      // bytes per porosity value
    size_t pop_bytes;  // one population buffer (q rows of p.P elements)
    size_t state_bytes;  // one snapshot (q rows of p.N elements)
    void* pop[2];
    void* dfield;
    bool own_mem;
    bool bound;
    bool porosity_set;
    int cur;           // buffer holding the current post-collision state
    // in-place (AA) pattern: one buffer (pop[0]); aa_pulled is set when it
    // holds the pulled populations of the next step in natural slots, clear
    // when it holds the post-collision populations in opposite slots
    bool aa;
    bool aa_pulled;
    long long step;
    hipStream_t stream;
    double* partials;  // FP64 per-block partials for the totals
    uint32_t partials_blocks;
    double* totals_dev;
    double* reduce_stage;  // first-pass results of the two-pass reduction
    int* flag_out;         // porosity check flag
    // batch of periodic boxes (hlbm_create_batch)
    bool batch;
    int n_items;
    int batch_mode;
    std::vector<hlbm::BatchItem> items;
    std::vector<char> item_porosity;
    hlbm::BatchItem* items_dev;
    uint32_t* tile_item_dev;
    double* tile_partials;
    double* item_totals_dev;
    unsigned long long* bar_sync;  // barrier arrivals and work counter
    int* bar_err;
    hlbm::BatchLaunch bl;
    hipGraphExec_t gexec[2];  // cached graph per starting buffer
    int gsteps[2];            // its step count (-1: none)
    int gkind[2];             // its kind: HLBM_BATCH_GRAPH or HLBM_BATCH_GRAPH_PERSISTENT
    std::vector<char> item_masked;  // items holding resolved obstacles (link mask rows in use)
    int n_masked;
    int cus;             // compute units of the device
    int batch_bpc;       // resident blocks per CU of the persistent kernel
    int max_blocks_per_cu;  // resident blocks of the persistent kernel that fit
    // adjoint tape (hlbm_set_tape): checkpoints of the state every `every`
    // steps since step `tape_origin`, replay states and segment records, and
    // two adjoint population buffers (FP64 for the FP64 form, FP32 otherwise)
    int tape_every;
    int tape_max;
    long long tape_origin;
    int tape_ncp;
    char* tape_cps;
    char* tape_seg;      // replay states: two sets (segments alternate between them) of two
                         // population buffers (the replay's sweeps alternate between them)
    char* tape_segrec;   // the replay's moment records: two sets of `every` steps of 4 rows of N
    // The forward steps of the tape's top two segments (the one holding step
    // max_steps and the one below it, one in each set) also write their moment
    // records, into their sets, so that a reverse sweep needs no replay of
    // them: tape_kept[k] says that set k holds the record of its segment
    // (kept_segment) from the segment's first step on.
    bool tape_kept[2];
    char* tape_lam[2];
    // HLBM_TAPE_MOMENTS: every recorded step also writes the pre-collision
    // moments of each cell (4 rows of N values in the adjoint's precision per
    // step), and the reverse sweep reads them instead of replaying segments
    // (no replay states)
    int tape_kind;
    char* tape_rec;
    // The reverse sweep replays the segment below the current one on a second
    // stream while the adjoint steps of the current one run on `stream`;
    // replayed[k] marks set k's replay done, consumed[k] the adjoint steps that
    // last read set k.
    hipStream_t tape_stream;
    hipEvent_t replayed[2];
    hipEvent_t consumed[2];
    // in-sweep diagnostics (hlbm_set_diagnostics): FP64 totals of the time
    // levels n with n % diag_every == 0, appended to a device log
    int diag_every;
    int diag_cap;
    int diag_count;
    long long diag_dropped;
    double* diag_log;
    std::vector<long long> diag_steps;
    // resolved solid cells (hlbm_set_solid_mask): per-cell link mask
    uint32_t* linkmask;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(HLBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(double s)
{
    if (!(s > 0.0) || !isfinite(s)) return false;
    int ex;
    double m = frexp(s, &ex);
    return m == 0.5;
}

// True when the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + nb && y < x + na;
}

// Copy q rows of `row` bytes between buffers whose rows are dpitch / spitch
// bytes apart (one 2D copy).
hipError_t copy_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t row, int q,
                     hipMemcpyKind kind, hipStream_t s)
{
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, row, (size_t)q, kind, s);
}

size_t elem_bytes(int storage)
{
    switch (storage) {
    case HLBM_F64: return 8;
    case HLBM_F32: return 4;
    case HLBM_F16S:
    case HLBM_BF16S: return 2;
    default: return 0;
    }
}

size_t porosity_elem_bytes(int storage)
{
    switch (storage) {
    case HLBM_F64: return 8;
    case HLBM_F32: return 4;
    case HLBM_F16S:
    case HLBM_BF16S: return 2;
    default: return 0;
    }
}

int porosity_rows(const hlbm_config* c) { return c->porosity_kind == HLBM_POROSITY_TENSOR ? 6 : 1; }

// Bytes of the porosity field: one dense row for a scalar control; six rows at
// the population row pitch for a tensor control.
size_t porosity_field_bytes(const hlbm_config* c, uint32_t n, uint32_t pitch)
{
    const size_t e = porosity_elem_bytes(c->storage);
    return porosity_rows(c) == 1 ? (size_t)n * e : 6 * (size_t)pitch * e;
}

int validate_config(const hlbm_config* c)
{
    if (!c) return fail(HLBM_EINVAL, "config is NULL");
    if (c->lattice != HLBM_D2Q9 && c->lattice != HLBM_D3Q19)
        return fail(HLBM_EINVAL, "lattice must be HLBM_D2Q9 or HLBM_D3Q19 (got %d)", c->lattice);
    if (elem_bytes(c->storage) == 0) return fail(HLBM_EINVAL, "unknown storage %d", c->storage);
    if (c->pattern != HLBM_AB && c->pattern != HLBM_AA)
        return fail(HLBM_EINVAL, "pattern must be HLBM_AB or HLBM_AA (got %d)", c->pattern);
    if (c->nx < 1 || c->ny < 1 || c->nz < 1)
        return fail(HLBM_EINVAL, "dimensions must be >= 1 (got %d x %d x %d)", c->nx, c->ny, c->nz);
    if (c->lattice == HLBM_D2Q9 && c->nz != 1) return fail(HLBM_EINVAL, "D2Q9 needs nz = 1");
    if (c->ny > 65535 || c->nz > 65535) return fail(HLBM_EUNSUPPORTED, "ny and nz must be <= 65535");
    const unsigned long long n = (unsigned long long)c->nx * c->ny * c->nz;
    if (n * elem_bytes(c->storage) >= (1ull << 32))
        return fail(HLBM_EUNSUPPORTED, "one population row (nx*ny*nz elements) must be < 4 GiB");
    if (!(c->tau > 0.5) || !isfinite(c->tau)) return fail(HLBM_EINVAL, "tau must be > 1/2 and finite");
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(c->force[a]) || !isfinite(c->inlet_u[a]))
            return fail(HLBM_EINVAL, "force and inlet_u must be finite");
        const int lo = c->bc_lo[a], hi = c->bc_hi[a];
        if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return fail(HLBM_EINVAL, "unknown face kind on axis %d", a);
        if ((lo == HLBM_PERIODIC) != (hi == HLBM_PERIODIC))
            return fail(HLBM_EINVAL, "axis %d: periodic must be on both sides or neither", a);
        const int n_a = a == 0 ? c->nx : (a == 1 ? c->ny : c->nz);
        if (lo != HLBM_PERIODIC && n_a < 3)
            return fail(HLBM_EINVAL, "axis %d: a non-periodic axis needs at least 3 cells", a);
    }
    if (c->lattice == HLBM_D2Q9 && (c->bc_lo[2] != HLBM_PERIODIC || c->force[2] != 0.0))
        return fail(HLBM_EINVAL, "D2Q9: z must be periodic and force[2] = 0");
    if (!(c->rho0 > 0.0) || !isfinite(c->rho0)) return fail(HLBM_EINVAL, "rho0 must be > 0");
    if (!(c->outlet_rho > 0.0) || !isfinite(c->outlet_rho))
        return fail(HLBM_EINVAL, "outlet_rho must be > 0");
    if ((c->storage == HLBM_F16S || c->storage == HLBM_BF16S) && !is_pow2(c->store_scale))
        return fail(HLBM_EINVAL, "store_scale must be a positive power of two");
    if (c->block_x != 0 && (c->block_x < 64 || c->block_x > 1024 || c->block_x % 64))
        return fail(HLBM_EINVAL, "block_x must be 0 or a multiple of 64 in [64, 1024]");
    if (c->porosity_kind != HLBM_POROSITY_SCALAR && c->porosity_kind != HLBM_POROSITY_TENSOR)
        return fail(HLBM_EINVAL, "unknown porosity_kind %d", c->porosity_kind);
    if (c->row_pad_bytes < 0 || c->row_pad_bytes > hlbm::ROW_PAD_MAX || c->row_pad_bytes % 256)
        return fail(HLBM_EINVAL, "row_pad_bytes must be a multiple of 256 in [0, %d]", hlbm::ROW_PAD_MAX);
    if (c->porosity_kind == HLBM_POROSITY_TENSOR && c->lattice != HLBM_D3Q19)
        return fail(HLBM_EUNSUPPORTED, "a tensor porosity control needs D3Q19");
    if (c->pattern == HLBM_AA) {
        // open faces need the cell's own post-collision state, whose slots the
        // neighbours are writing during the shifted step
        for (int a = 0; a < 3; ++a)
            if ((c->bc_lo[a] != HLBM_PERIODIC && c->bc_lo[a] != HLBM_WALL) ||
                (c->bc_hi[a] != HLBM_PERIODIC && c->bc_hi[a] != HLBM_WALL))
                return fail(HLBM_EUNSUPPORTED,
                            "the in-place pattern (HLBM_AA) takes periodic and wall faces only (no open faces)");
        if (c->block_x > 256) return fail(HLBM_EUNSUPPORTED, "the in-place pattern (HLBM_AA) needs block_x <= 256");
    }
    return HLBM_OK;
}

void fill_params(const hlbm_config* c, Params* p)
{
    memset(p, 0, sizeof(*p));
    p->nx = c->nx;
    p->ny = c->ny;
    p->nz = c->nz;
    p->N = (uint32_t)((unsigned long long)c->nx * c->ny * c->nz);
    p->P = hlbm::row_pitch(p->N, elem_bytes(c->storage), c->row_pad_bytes);
    p->omega = 1.0 / c->tau;
    p->pref = 1.0 - 0.5 / c->tau;
    for (int a = 0; a < 3; ++a) {
        p->F[a] = c->force[a];
        p->bc_lo[a] = c->bc_lo[a];
        p->bc_hi[a] = c->bc_hi[a];
        p->inlet_u[a] = c->inlet_u[a];
    }
    p->rho0 = c->rho0;
    const bool s16 = c->storage == HLBM_F16S || c->storage == HLBM_BF16S;
    p->scale = s16 ? c->store_scale : 1.0;
    p->inv_scale = 1.0 / p->scale;
    p->outlet_rho = c->outlet_rho;
}

int auto_block_x(int nx)
{
    int b = ((nx + 63) / 64) * 64;
    if (b > 256) b = 256;
    return b;
}

// Sweep / moments mode of an in-place context: the local step when the buffer
// holds pulled populations, the shifted step otherwise; wall variants when a
// face is a wall.
int aa_mode(const hlbm_ctx* c)
{
    const bool walls = c->bcmode != hlbm::BC_PERIODIC;
    if (c->aa_pulled) return walls ? hlbm::BC_AA_EVEN_W : hlbm::BC_AA_EVEN;
    return walls ? hlbm::BC_AA_ODD_W : hlbm::BC_AA_ODD;
}

int check_ctx(const hlbm_ctx* c)
{
    if (!c) return fail(HLBM_EINVAL, "context is NULL");
    return HLBM_OK;
}

int ensure_partials(hlbm_ctx* c, uint32_t nblocks)
{
    if (c->partials && c->partials_blocks >= nblocks) return HLBM_OK;
    if (c->partials) (void)hipFree(c->partials);
    c->partials = nullptr;
    c->partials_blocks = 0;
    hipError_t e = hipMalloc(&c->partials, sizeof(double) * 4 * (size_t)nblocks);
    if (e != hipSuccess) return fail(HLBM_ENOMEM, "partials allocation: %s", hipGetErrorString(e));
    c->partials_blocks = nblocks;
    return HLBM_OK;
}

int zero_state(hlbm_ctx* c)
{
    for (int k = 0; k < (c->aa ? 1 : 2); ++k) {
        hipError_t e = hipMemsetAsync(c->pop[k], 0, c->pop_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "zeroing populations");
    }
    c->cur = 0;
    c->aa_pulled = false;  // zeros are the post-collision state in any slot order
    c->step = 0;
    return HLBM_OK;
}

// State of an in-place context in A/B layout (the post-collision populations
// of the last step, population i of cell x at row i, element x).
int aa_get_state(hlbm_ctx* c, void* dst, int on_device, long long* step)
{
    hipError_t e = hipSuccess;
    const size_t row = (size_t)c->p.N * c->elem, pitch = (size_t)c->p.P * c->elem;
    void* tmp = nullptr;
    if (!c->aa_pulled && !on_device) {
        // opposite slots: one row copy per population
        for (int i = 0; i < c->q && e == hipSuccess; ++i)
            e = hipMemcpyAsync(static_cast<char*>(dst) + (size_t)i * row,
                               static_cast<const char*>(c->pop[0]) + (size_t)hlbm::opposite(i) * pitch, row,
                               hipMemcpyDeviceToHost, c->stream);
    } else {
        void* out = dst;
        if (!on_device) {
            e = hipMalloc(&tmp, c->state_bytes);
            if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
            out = tmp;
        } else if (overlaps(dst, c->state_bytes, c->pop[0], c->pop_bytes)) {
            return fail(HLBM_EINVAL, "dst overlaps the population buffer");
        }
        e = hlbm::launch_aa_export(c->q, c->cfg.storage, c->p, c->pop[0], out, c->aa_pulled ? 0 : 1, c->stream);
        if (e == hipSuccess && tmp) e = hipMemcpyAsync(dst, tmp, c->state_bytes, hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "get_state");
    if (step) *step = c->step;
    return HLBM_OK;
}

void tape_free(hlbm_ctx* c)
{
    if (c->tape_stream) (void)hipStreamSynchronize(c->tape_stream);
    if (c->tape_cps) (void)hipFree(c->tape_cps);
    if (c->tape_seg) (void)hipFree(c->tape_seg);
    if (c->tape_segrec) (void)hipFree(c->tape_segrec);
    c->tape_segrec = nullptr;
    for (int k = 0; k < 2; ++k) {
        if (c->replayed[k]) (void)hipEventDestroy(c->replayed[k]);
        if (c->consumed[k]) (void)hipEventDestroy(c->consumed[k]);
        c->replayed[k] = c->consumed[k] = nullptr;
    }
    if (c->tape_stream) (void)hipStreamDestroy(c->tape_stream);
    c->tape_stream = nullptr;
    for (int k = 0; k < 2; ++k)
        if (c->tape_lam[k]) (void)hipFree(c->tape_lam[k]);
    if (c->tape_rec) (void)hipFree(c->tape_rec);
    c->tape_rec = nullptr;
    c->tape_cps = nullptr;
    c->tape_seg = nullptr;
    c->tape_lam[0] = c->tape_lam[1] = nullptr;
    c->tape_every = 0;
    c->tape_max = 0;
    c->tape_ncp = 0;
}

// Bytes of one step of a moment record: 4 rows of N values in the adjoint's
// precision (FP64 for the FP64 form, FP32 otherwise).
size_t record_step_bytes(const hlbm_ctx* c)
{
    return 4 * (size_t)c->p.N * hlbm::adjoint_elem_bytes(c->cfg.storage);
}

// The segment whose record the forward steps keep in replay set k: the
// highest segment of parity k up to the top one, -1 if there is none.
static long long kept_segment(const hlbm_ctx* c, int k)
{
    const long long mtop = (c->tape_max - 1) / c->tape_every;
    return ((mtop & 1) == k) ? mtop : mtop - 1;
}

// Bytes of a moment record of `steps` steps.
size_t tape_record_bytes(const hlbm_ctx* c, int steps) { return (size_t)steps * record_step_bytes(c); }

// Start recording at the current state: checkpoint 0 is the current state.
int tape_restart(hlbm_ctx* c)
{
    if (!c->tape_every) return HLBM_OK;
    c->tape_origin = c->step;
    c->tape_kept[0] = c->tape_kept[1] = false;
    hipError_t e = hipMemcpyAsync(c->tape_cps, c->pop[c->cur], c->pop_bytes, hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(e, "tape checkpoint");
    return HLBM_OK;
}

// Resident grid and chunk of the persistent kernel (0 = default); drops the
// cached graphs, which hold the old launch shape.
void set_batch_schedule(hlbm_ctx* c, int blocks_per_cu, int chunk)
{
    if (blocks_per_cu == 0) {
        blocks_per_cu = hlbm::BATCH_THREADS_PER_CU_DEFAULT / (int)c->bl.tile;
        if (blocks_per_cu < 1) blocks_per_cu = 1;
        if (blocks_per_cu > c->max_blocks_per_cu) blocks_per_cu = c->max_blocks_per_cu;
    }
    long long grid = (long long)blocks_per_cu * c->cus;
    if (grid > (long long)c->bl.ntiles) grid = (long long)c->bl.ntiles;
    if (grid < 1) grid = 1;
    c->bl.grid = (int)grid;
    c->bl.chunk = (uint32_t)(chunk ? chunk : hlbm::CHUNK_DEFAULT);
    c->batch_bpc = blocks_per_cu;
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
        c->gsteps[k] = -1;
    }
}

int batch_check_barrier(hlbm_ctx* c)
{
    int err = 0;
    hipError_t e = hipMemcpy(&err, c->bar_err, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the barrier flag");
    if (err) return fail(HLBM_EDEVICE, "a grid barrier of the persistent batch kernel timed out");
    return HLBM_OK;
}

int batch_step(hlbm_ctx* c, int nsteps)
{
    if (nsteps == 0) return HLBM_OK;
    hipError_t e = hipSuccess;
    const int storage = c->cfg.storage;
    if (c->batch_mode == HLBM_BATCH_PER_STEP) {
        for (int t = 0; t < nsteps && e == hipSuccess; ++t) {
            e = hlbm::launch_batch_step(storage, c->bl, c->pop[c->cur], c->pop[c->cur ^ 1], c->dfield,
                                        c->stream);
            if (e == hipSuccess) c->cur ^= 1;
        }
    } else if (c->batch_mode == HLBM_BATCH_PERSISTENT) {
        e = hlbm::launch_batch_persistent(storage, c->bl, c->pop[0], c->pop[1], c->dfield, nsteps, c->cur,
                                          c->stream);
        if (e == hipSuccess) c->cur ^= (nsteps & 1);
    } else {
        const int k = c->cur;
        const int kind = c->batch_mode;
        if (!c->gexec[k] || c->gsteps[k] != nsteps || c->gkind[k] != kind) {
            if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
            c->gexec[k] = nullptr;
            c->gsteps[k] = -1;
            e = hlbm::build_batch_graph(storage, c->bl, c->pop[0], c->pop[1], c->dfield, nsteps, k,
                                        kind == HLBM_BATCH_GRAPH_PERSISTENT, &c->gexec[k]);
            if (e != hipSuccess) return hip_fail(e, "building the batch graph");
            c->gsteps[k] = nsteps;
            c->gkind[k] = kind;
        }
        e = hipGraphLaunch(c->gexec[k], c->stream);
        if (e == hipSuccess) c->cur ^= (nsteps & 1);
    }
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    c->step += nsteps;
    return HLBM_OK;
}

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];

int scratch_address(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "moments_noalloc: current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(HLBM_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "moments_noalloc: address of the static scratch");
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return HLBM_OK;
}

}  // namespace

extern "C" {

int hlbm_version(void) { return HLBM_ABI_VERSION; }

const char* hlbm_last_error(void) { return g_err; }

int hlbm_config_default(hlbm_config* cfg)
{
    if (!cfg) return fail(HLBM_EINVAL, "config is NULL");
    memset(cfg, 0, sizeof(*cfg));
    cfg->lattice = HLBM_D3Q19;
    cfg->storage = HLBM_F32;
    cfg->pattern = HLBM_AB;
    cfg->nx = cfg->ny = cfg->nz = 32;
    cfg->tau = 0.6;
    cfg->outlet_rho = 1.0;
    cfg->rho0 = 1.0;
    cfg->store_scale = 1.0;
    return HLBM_OK;
}

int hlbm_lattice_info(int lattice, int* c, double* w)
{
    if (!c || !w) return fail(HLBM_EINVAL, "NULL output");
    if (lattice == HLBM_D2Q9) {
        for (int i = 0; i < 9; ++i) {
            c[3 * i] = hlbm::D2Q9::cx[i];
            c[3 * i + 1] = hlbm::D2Q9::cy[i];
            c[3 * i + 2] = hlbm::D2Q9::cz[i];
            w[i] = hlbm::D2Q9::w[i];
        }
        return HLBM_OK;
    }
    if (lattice == HLBM_D3Q19) {
        for (int i = 0; i < 19; ++i) {
            c[3 * i] = hlbm::D3Q19::cx[i];
            c[3 * i + 1] = hlbm::D3Q19::cy[i];
            c[3 * i + 2] = hlbm::D3Q19::cz[i];
            w[i] = hlbm::D3Q19::w[i];
        }
        return HLBM_OK;
    }
    return fail(HLBM_EINVAL, "unknown lattice %d", lattice);
}

int hlbm_required_bytes(const hlbm_config* cfg, size_t* pop_bytes, size_t* porosity_bytes)
{
    int rc = validate_config(cfg);
    if (rc) return rc;
    const size_t n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    const size_t pitch = hlbm::row_pitch((uint32_t)n, elem_bytes(cfg->storage), cfg->row_pad_bytes);
    if (pop_bytes) *pop_bytes = pitch * (size_t)cfg->lattice * elem_bytes(cfg->storage);
    if (porosity_bytes) *porosity_bytes = porosity_field_bytes(cfg, (uint32_t)n, (uint32_t)pitch);
    return HLBM_OK;
}

int hlbm_create(const hlbm_config* cfg, hlbm_ctx** out)
{
    if (!out) return fail(HLBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc) return rc;
    hlbm_ctx* c = new (std::nothrow) hlbm_ctx();
    if (!c) return fail(HLBM_ENOMEM, "host allocation of the context failed");
    c->cfg = *cfg;
    fill_params(cfg, &c->p);
    c->q = cfg->lattice;
    c->aa = cfg->pattern == HLBM_AA;
    bool general = false;
    for (int a = 0; a < 3; ++a)
        if (cfg->bc_lo[a] != HLBM_PERIODIC) general = true;
    c->bcmode = general ? hlbm::BC_GENERAL : hlbm::BC_PERIODIC;
    c->bx = cfg->block_x ? cfg->block_x : auto_block_x(cfg->nx);
    c->elem = elem_bytes(cfg->storage);
    c->delem = porosity_elem_bytes(cfg->storage);
    c->pop_bytes = (size_t)c->p.P * (size_t)c->q * c->elem;
    c->state_bytes = (size_t)c->p.N * (size_t)c->q * c->elem;
    c->stream = static_cast<hipStream_t>(cfg->hip_stream);
    c->own_mem = !cfg->external_memory;
    if (c->own_mem) {
        hipError_t e = hipMalloc(&c->pop[0], c->pop_bytes);
        if (e == hipSuccess && !c->aa) e = hipMalloc(&c->pop[1], c->pop_bytes);
        if (e == hipSuccess) e = hipMalloc(&c->dfield, porosity_field_bytes(cfg, c->p.N, c->p.P));
        if (e != hipSuccess) {
            hlbm_destroy(c);
            return fail(HLBM_ENOMEM, "device allocation of %zu bytes per buffer failed: %s",
                        c->pop_bytes, hipGetErrorString(e));
        }
        c->bound = true;
        rc = zero_state(c);
        if (rc) {
            hlbm_destroy(c);
            return rc;
        }
    }
    hipError_t e = hipMalloc(&c->flag_out, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->totals_dev, 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->reduce_stage, 4 * sizeof(double) * hlbm::REDUCE_STAGE);
    if (e != hipSuccess) {
        hlbm_destroy(c);
        return fail(HLBM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    rc = ensure_partials(c, hlbm::cell_launch(c->p, c->bx).nblocks);
    if (rc) {
        hlbm_destroy(c);
        return rc;
    }
    *out = c;
    return HLBM_OK;
}

int hlbm_bind_buffers(hlbm_ctx* c, void* pop_a, void* pop_b, void* porosity)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->own_mem) return fail(HLBM_ESTATE, "context owns its memory (external_memory = 0)");
    if (c->aa && pop_b) return fail(HLBM_EINVAL, "the in-place pattern takes one population buffer (pop_b = NULL)");
    if (!pop_a || (!c->aa && !pop_b) || !porosity) return fail(HLBM_EINVAL, "NULL buffer");
    if (pop_a == pop_b) return fail(HLBM_EINVAL, "population buffers must differ");
    if (((uintptr_t)pop_a | (uintptr_t)pop_b | (uintptr_t)porosity) & 255u)
        return fail(HLBM_EINVAL, "buffers must be 256-byte aligned");
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->dfield = porosity;
    c->bound = true;
    c->porosity_set = false;
    rc = zero_state(c);
    if (rc) return rc;
    return tape_restart(c);
}

int hlbm_destroy(hlbm_ctx* c)
{
    if (!c) return HLBM_OK;
    int rc = HLBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(e, "destroy: outstanding work failed");
    if (c->own_mem) {
        if (c->pop[0]) (void)hipFree(c->pop[0]);
        if (c->pop[1]) (void)hipFree(c->pop[1]);
        if (c->dfield) (void)hipFree(c->dfield);
    }
    if (c->partials) (void)hipFree(c->partials);
    if (c->totals_dev) (void)hipFree(c->totals_dev);
    if (c->reduce_stage) (void)hipFree(c->reduce_stage);
    if (c->flag_out) (void)hipFree(c->flag_out);
    if (c->diag_log) (void)hipFree(c->diag_log);
    if (c->linkmask) (void)hipFree(c->linkmask);
    for (int k = 0; k < 2; ++k)
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    tape_free(c);
    if (c->items_dev) (void)hipFree(c->items_dev);
    if (c->tile_item_dev) (void)hipFree(c->tile_item_dev);
    if (c->tile_partials) (void)hipFree(c->tile_partials);
    if (c->item_totals_dev) (void)hipFree(c->item_totals_dev);
    if (c->bar_sync) (void)hipFree(c->bar_sync);
    if (c->bar_err) (void)hipFree(c->bar_err);
    delete c;
    return rc;
}

int hlbm_set_porosity(hlbm_ctx* c, const void* d, int dtype, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "use hlbm_batch_set_porosity for a batch");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!d) return fail(HLBM_EINVAL, "porosity array is NULL");
    if (dtype < HLBM_DT_F64 || dtype > HLBM_DT_F16) return fail(HLBM_EINVAL, "unknown dtype %d", dtype);
    const size_t in_elem = dtype == HLBM_DT_F64 ? 8 : (dtype == HLBM_DT_F32 ? 4 : 2);
    const size_t n = c->p.N;
    const size_t rows = porosity_rows(&c->cfg);
    const void* src = d;
    void* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
        e = hipMalloc(&tmp, rows * n * in_elem);
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        e = hipMemcpyAsync(tmp, d, rows * n * in_elem, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return hip_fail(e, "porosity upload");
        }
        src = tmp;
    }
    e = hlbm::launch_porosity_convert(dtype, src, c->cfg.storage, c->cfg.porosity_kind, c->dfield, (uint32_t)n, c->p.P,
                                      c->flag_out,
                                      c->stream);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, c->flag_out, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "porosity conversion");
    if (flag) {
        c->porosity_set = false;
        return fail(HLBM_EINVAL, rows == 1 ? "porosity values must be finite and in [0, 1]"
                                           : "porosity tensors must be finite with eigenvalues in [0, 1]");
    }
    c->porosity_set = true;
    return tape_restart(c);
}

int hlbm_step(hlbm_ctx* c, int nsteps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(HLBM_EINVAL, "nsteps must be >= 0");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!c->porosity_set) return fail(HLBM_ESTATE, "porosity not set");
    if (c->batch) return batch_step(c, nsteps);
    if (c->tape_every && c->step - c->tape_origin + nsteps > c->tape_max)
        return fail(HLBM_EINVAL, "the tape holds %d steps; %lld recorded, %d more requested", c->tape_max,
                    c->step - c->tape_origin, nsteps);
    for (int t = 0; t < nsteps; ++t) {
        hipError_t e;
        char* mrec = nullptr;  // this step's moment record (HLBM_TAPE_MOMENTS)
        if (c->tape_every) {
            const long long rel = c->step - c->tape_origin;
            if (rel > 0 && rel % c->tape_every == 0) {
                e = hipMemcpyAsync(c->tape_cps + (size_t)(rel / c->tape_every) * c->pop_bytes, c->pop[c->cur],
                                   c->pop_bytes, hipMemcpyDeviceToDevice, c->stream);
                if (e != hipSuccess) return hip_fail(e, "tape checkpoint");
            }
            if (c->tape_rec) {
                mrec = c->tape_rec + (size_t)rel * record_step_bytes(c);
            } else if (c->tape_segrec) {
                // forward step rel + 1 of segment m, one of the top two: its
                // moment record, as the replay would write it (record j = step
                // mK + j + 1)
                const long long K = c->tape_every, m = rel / K;
                const int k = (int)(m & 1);
                if (m == kept_segment(c, k)) {
                    mrec = c->tape_segrec + ((size_t)k * (size_t)K + (size_t)(rel - m * K)) * record_step_bytes(c);
                    if (rel == m * K) c->tape_kept[k] = true;
                }
            }
        }
        const bool diag = c->diag_every && c->step % c->diag_every == 0;
        const bool record = diag && c->diag_count < c->diag_cap;
        if (diag && !record) c->diag_dropped += 1;
        if (c->aa) {
            e = hlbm::launch_sweep(c->q, c->cfg.storage, aa_mode(c), c->cfg.porosity_kind, c->p, c->pop[0], c->pop[0], c->dfield, c->bx, c->stream,
                                   record ? c->partials : nullptr);
        } else if (mrec) {
            // a recording step: the diagnostics' partials, if due, from the
            // moments kernel (the same arithmetic as the diagnostic sweep)
            e = hipSuccess;
            if (record)
                e = hlbm::launch_moments(c->q, c->cfg.storage, c->bcmode, c->p, c->pop[c->cur], nullptr, nullptr, 1,
                                         c->partials, c->bx, c->stream);
            if (e == hipSuccess)
                e = hlbm::launch_sweep(c->q, c->cfg.storage, c->bcmode, c->cfg.porosity_kind, c->p, c->pop[c->cur],
                                       c->pop[c->cur ^ 1], c->dfield, c->bx, c->stream, nullptr, mrec);
        } else {
            e = hlbm::launch_sweep(c->q, c->cfg.storage, c->bcmode, c->cfg.porosity_kind, c->p, c->pop[c->cur],
                                   c->pop[c->cur ^ 1], c->dfield, c->bx, c->stream, record ? c->partials : nullptr);
        }
        if (e == hipSuccess && record)
            e = hlbm::launch_reduce4(c->partials, hlbm::cell_launch(c->p, c->bx).nblocks, c->reduce_stage,
                                     c->diag_log + 4 * (size_t)c->diag_count, c->stream);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
        if (record) {
            c->diag_steps.push_back(c->step);
            c->diag_count += 1;
        }
        if (c->aa)
            c->aa_pulled = !c->aa_pulled;
        else
            c->cur ^= 1;
        c->step += 1;
    }
    return HLBM_OK;
}

int hlbm_get_step(const hlbm_ctx* c, long long* step)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!step) return fail(HLBM_EINVAL, "step is NULL");
    *step = c->step;
    return HLBM_OK;
}

int hlbm_moments(hlbm_ctx* c, void* drho, void* u, int dtype, int on_device, double* totals)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "use hlbm_batch_moments for a batch");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (dtype != HLBM_DT_F64 && dtype != HLBM_DT_F32) return fail(HLBM_EINVAL, "dtype must be F64 or F32");
    const size_t osz = dtype == HLBM_DT_F64 ? 8 : 4;
    const size_t n = c->p.N;
    void* ddr = drho;
    void* du = u;
    void* tmp = nullptr;
    hipError_t e;
    if (!on_device && (drho || u)) {
        e = hipMalloc(&tmp, 4 * n * osz);
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        ddr = drho ? tmp : nullptr;
        du = u ? static_cast<char*>(tmp) + n * osz : nullptr;
    }
    const hlbm::Launch l = hlbm::cell_launch(c->p, c->bx);
    double* partials = nullptr;
    if (totals) {
        rc = ensure_partials(c, l.nblocks);
        if (rc) {
            if (tmp) (void)hipFree(tmp);
            return rc;
        }
        partials = c->partials;
    }
    const int mbc = c->aa ? aa_mode(c) : c->bcmode;
    e = hlbm::launch_moments(c->q, c->cfg.storage, mbc, c->p, c->pop[c->cur], ddr, du,
                             dtype == HLBM_DT_F64, partials, c->bx, c->stream);
    if (e == hipSuccess && totals)
        e = hlbm::launch_reduce4(partials, l.nblocks, c->reduce_stage, c->totals_dev, c->stream);
    if (e == hipSuccess && totals)
        e = hipMemcpyAsync(totals, c->totals_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && tmp && drho)
        e = hipMemcpyAsync(drho, ddr, n * osz, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && tmp && u)
        e = hipMemcpyAsync(u, du, 3 * n * osz, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "moments");
    if (totals)
        for (int k = 0; k < 4; ++k)
            if (!isfinite(totals[k])) return fail(HLBM_ENUMERIC, "non-finite total (component %d)", k);
    return HLBM_OK;
}

int hlbm_moments_noalloc(hlbm_ctx* c, void* drho, void* u, int dtype, double* totals)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "moments_noalloc takes a single context, not a batch");
    if (dtype != HLBM_DT_F64 && dtype != HLBM_DT_F32) return fail(HLBM_EINVAL, "dtype must be F64 or F32");
    const hlbm::Launch l = hlbm::cell_launch(c->p, c->bx);
    if (totals && l.nblocks > kScratchBlocks)
        return fail(HLBM_EINVAL, "totals of %u blocks exceed the static scratch (%u blocks of block_x cells)",
                    l.nblocks, kScratchBlocks);
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    double* sc = nullptr;
    if (totals) {
        rc = scratch_address(&sc);
        if (rc) return rc;
    }
    double* partials = sc;
    double* stage = sc ? sc + 4 * (size_t)kScratchBlocks : nullptr;
    const int mbc = c->aa ? aa_mode(c) : c->bcmode;
    hipError_t e = hlbm::launch_moments(c->q, c->cfg.storage, mbc, c->p, c->pop[c->cur], drho, u,
                                        dtype == HLBM_DT_F64, partials, c->bx, c->stream);
    if (e == hipSuccess && totals) e = hlbm::launch_reduce4(partials, l.nblocks, stage, totals, c->stream);
    if (e != hipSuccess) return hip_fail(e, "moments_noalloc launch");
    return HLBM_OK;
}

int hlbm_state_bytes(const hlbm_ctx* c, size_t* bytes)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!bytes) return fail(HLBM_EINVAL, "bytes is NULL");
    *bytes = c->state_bytes;
    return HLBM_OK;
}

int hlbm_get_state(hlbm_ctx* c, void* dst, int on_device, long long* step)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!dst) return fail(HLBM_EINVAL, "dst is NULL");
    if (c->aa) return aa_get_state(c, dst, on_device, step);
    if (on_device && overlaps(dst, c->state_bytes, c->pop[c->cur], c->pop_bytes))
        return fail(HLBM_EINVAL, "dst overlaps the current population buffer");
    const size_t row = (size_t)c->p.N * c->elem;
    hipError_t e = copy_rows(dst, row, c->pop[c->cur], (size_t)c->p.P * c->elem, row, c->q,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "get_state");
    if (step) *step = c->step;
    return HLBM_OK;
}

int hlbm_set_state(hlbm_ctx* c, const void* src, int on_device, long long step)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!src) return fail(HLBM_EINVAL, "src is NULL");
    if (step < 0) return fail(HLBM_EINVAL, "step must be >= 0");
    hipError_t e = hipSuccess;
    if (c->aa) {
        if (on_device && overlaps(src, c->state_bytes, c->pop[0], c->pop_bytes))
            return fail(HLBM_EINVAL, "src overlaps the population buffer");
        // row i of the A/B-layout state into slot row opp(i): ready for the
        // shifted step
        const size_t row = (size_t)c->p.N * c->elem, pitch = (size_t)c->p.P * c->elem;
        for (int i = 0; i < c->q && e == hipSuccess; ++i)
            e = hipMemcpyAsync(static_cast<char*>(c->pop[0]) + (size_t)hlbm::opposite(i) * pitch,
                               static_cast<const char*>(src) + (size_t)i * row, row,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
        c->aa_pulled = false;
    } else {
        if (on_device && overlaps(src, c->state_bytes, c->pop[c->cur], c->pop_bytes))
            return fail(HLBM_EINVAL, "src overlaps the current population buffer");
        const size_t row = (size_t)c->p.N * c->elem;
        e = copy_rows(c->pop[c->cur], (size_t)c->p.P * c->elem, src, row, row, c->q,
                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    c->step = step;
    return tape_restart(c);
}

int hlbm_reset(hlbm_ctx* c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    rc = zero_state(c);
    if (rc) return rc;
    return tape_restart(c);
}

int hlbm_set_diagnostics(hlbm_ctx* c, int every, int capacity)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "use hlbm_batch_moments for a batch");
    if (every < 0 || capacity < 0) return fail(HLBM_EINVAL, "every and capacity must be >= 0");
    if (every > 0 && capacity < 1) return fail(HLBM_EINVAL, "capacity must be >= 1");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set_diagnostics: outstanding work failed");
    if (c->diag_log) (void)hipFree(c->diag_log);
    c->diag_log = nullptr;
    c->diag_every = 0;
    c->diag_cap = 0;
    c->diag_count = 0;
    c->diag_dropped = 0;
    c->diag_steps.clear();
    if (every == 0) return HLBM_OK;
    e = hipMalloc(&c->diag_log, 4 * sizeof(double) * (size_t)capacity);
    if (e != hipSuccess) return fail(HLBM_ENOMEM, "diagnostics log: %s", hipGetErrorString(e));
    c->diag_every = every;
    c->diag_cap = capacity;
    return ensure_partials(c, hlbm::cell_launch(c->p, c->bx).nblocks);
}

int hlbm_read_diagnostics(hlbm_ctx* c, double* out, int max_records, int* count, long long* dropped)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!count) return fail(HLBM_EINVAL, "count is NULL");
    if (max_records < 0 || (max_records > 0 && !out)) return fail(HLBM_EINVAL, "bad output array");
    const int n = c->diag_count < max_records ? c->diag_count : max_records;
    std::vector<double> tmp(4 * (size_t)(n > 0 ? n : 1));
    hipError_t e = hipSuccess;
    if (n > 0)
        e = hipMemcpyAsync(tmp.data(), c->diag_log, 4 * sizeof(double) * (size_t)n, hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "read_diagnostics");
    for (int k = 0; k < n; ++k) {
        out[5 * k] = (double)c->diag_steps[k];
        for (int j = 0; j < 4; ++j) {
            out[5 * k + 1 + j] = tmp[4 * (size_t)k + j];
            if (!isfinite(tmp[4 * (size_t)k + j])) rc = HLBM_ENUMERIC;
        }
    }
    *count = n;
    if (dropped) *dropped = c->diag_dropped + (c->diag_count - n);
    c->diag_count = 0;
    c->diag_dropped = 0;
    c->diag_steps.clear();
    if (rc) return fail(rc, "a diagnostic total is not finite");
    return HLBM_OK;
}

int hlbm_set_solid_mask(hlbm_ctx* c, const unsigned char* mask, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "batch items take no solid mask");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    for (int a = 0; a < 3; ++a)
        if (c->cfg.bc_lo[a] != HLBM_PERIODIC)
            return fail(HLBM_EUNSUPPORTED, "a solid mask needs periodic faces on every axis");
    if (c->aa) return fail(HLBM_EUNSUPPORTED, "a solid mask needs the two-buffer pattern (HLBM_AB)");
    if (c->tape_every) return fail(HLBM_ESTATE, "free the adjoint tape first (hlbm_set_tape(ctx, 0, 0))");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set_solid_mask: outstanding work failed");
    if (!mask) {
        c->bcmode = hlbm::BC_PERIODIC;
        c->p.linkmask = nullptr;
        return HLBM_OK;
    }
    const size_t n = c->p.N;
    if (!c->linkmask) {
        e = hipMalloc(&c->linkmask, n * sizeof(uint32_t));
        if (e != hipSuccess) {
            c->linkmask = nullptr;
            return fail(HLBM_ENOMEM, "link mask allocation: %s", hipGetErrorString(e));
        }
    }
    const unsigned char* src = mask;
    void* tmp = nullptr;
    if (!on_device) {
        e = hipMalloc(&tmp, n);
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        e = hipMemcpyAsync(tmp, mask, n, hipMemcpyHostToDevice, c->stream);
        src = static_cast<const unsigned char*>(tmp);
    }
    if (e == hipSuccess) e = hlbm::launch_linkmask(c->q, c->p, src, c->linkmask, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "solid mask");
    c->bcmode = hlbm::BC_MASKED;
    c->p.linkmask = c->linkmask;
    return HLBM_OK;
}

int hlbm_set_tape(hlbm_ctx* c, int every, int max_steps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "a batch has no adjoint");
    if (c->bcmode == hlbm::BC_MASKED)
        return fail(HLBM_EUNSUPPORTED, "the adjoint does not cover resolved solid cells");
    if (c->aa) return fail(HLBM_EUNSUPPORTED, "the adjoint tape needs the two-buffer pattern (HLBM_AB)");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (every < 0 || max_steps < 0) return fail(HLBM_EINVAL, "every and max_steps must be >= 0");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set_tape: outstanding work failed");
    // The tape it already has (same every, max_steps and kind), as in a loop
    // of forward and reverse sweeps: its memory, stream and events are kept,
    // and recording restarts at the current state.
    const bool have = c->tape_kind == HLBM_TAPE_MOMENTS ? c->tape_rec != nullptr : c->tape_segrec != nullptr;
    if (every != 0 && every == c->tape_every && max_steps == c->tape_max && have) {
        e = hipStreamSynchronize(c->tape_stream);
        if (e != hipSuccess) return hip_fail(e, "set_tape: outstanding replays failed");
        return tape_restart(c);
    }
    tape_free(c);
    if (every == 0) return HLBM_OK;
    const size_t lam_elem = hlbm::adjoint_elem_bytes(c->cfg.storage);
    if ((unsigned long long)c->p.N * lam_elem >= (1ull << 32))
        return fail(HLBM_EUNSUPPORTED, "an adjoint population row (nx*ny*nz elements) must be < 4 GiB");
    const int ncp = max_steps / every + 1;
    // adjoint rows take the population row pitch P (in elements of the adjoint type)
    const size_t lam_bytes = (size_t)c->p.P * (size_t)c->q * lam_elem;
    const bool rec = c->tape_kind == HLBM_TAPE_MOMENTS;
    e = hipMalloc(&c->tape_cps, (size_t)ncp * c->pop_bytes);
    if (e == hipSuccess && !rec) e = hipMalloc(&c->tape_seg, 4 * c->pop_bytes);
    if (e == hipSuccess && !rec) e = hipMalloc((void**)&c->tape_segrec, 2 * tape_record_bytes(c, every));
    if (e == hipSuccess && rec) e = hipMalloc((void**)&c->tape_rec, tape_record_bytes(c, max_steps));
    if (e == hipSuccess) e = hipMalloc(&c->tape_lam[0], lam_bytes);
    if (e == hipSuccess) e = hipMalloc(&c->tape_lam[1], lam_bytes);
    // default priority (a stream of another priority is never used here)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->tape_stream, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&c->replayed[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->consumed[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        tape_free(c);
        return fail(HLBM_ENOMEM, "tape allocation (%d checkpoints of %zu bytes): %s", ncp, c->pop_bytes,
                    hipGetErrorString(e));
    }
    c->tape_every = every;
    c->tape_max = max_steps;
    c->tape_ncp = ncp;
    return tape_restart(c);
}

int hlbm_set_tape_kind(hlbm_ctx* c, int kind)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "a batch has no adjoint");
    if (kind != HLBM_TAPE_REPLAY && kind != HLBM_TAPE_MOMENTS) return fail(HLBM_EINVAL, "unknown tape kind %d", kind);
    if (kind == c->tape_kind) return HLBM_OK;
    c->tape_kind = kind;
    // a tape in use is rebuilt in the new kind and restarts at the current state
    if (c->tape_every) return hlbm_set_tape(c, c->tape_every, c->tape_max);
    return HLBM_OK;
}

int hlbm_tape_info(const hlbm_ctx* c, int* every, int* max_steps, long long* recorded, size_t* device_bytes)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (every) *every = c->tape_every;
    if (max_steps) *max_steps = c->tape_max;
    if (recorded) *recorded = c->tape_every ? c->step - c->tape_origin : 0;
    if (device_bytes) {
        size_t b = 0;
        if (c->tape_every) {
            const bool rec = c->tape_kind == HLBM_TAPE_MOMENTS;
            b = ((size_t)c->tape_ncp + (rec ? 0 : 4)) * c->pop_bytes +
                2 * (size_t)c->p.P * (size_t)c->q * hlbm::adjoint_elem_bytes(c->cfg.storage) +
                (rec ? tape_record_bytes(c, c->tape_max) : 2 * tape_record_bytes(c, c->tape_every));
        }
        *device_bytes = b;
    }
    return HLBM_OK;
}

int hlbm_adjoint_step(hlbm_ctx* c, int nsteps, const double* dJ_drho, const double* dJ_du, double* dJ_dd,
                      int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->batch) return fail(HLBM_EUNSUPPORTED, "a batch has no adjoint");
    if (!c->tape_every) return fail(HLBM_ESTATE, "no tape: call hlbm_set_tape before the forward steps");
    if (!c->porosity_set) return fail(HLBM_ESTATE, "porosity not set");
    if (!dJ_drho || !dJ_du || !dJ_dd) return fail(HLBM_EINVAL, "NULL cotangent or gradient array");
    const long long R0 = c->step - c->tape_origin;
    if (nsteps < 0 || nsteps > R0)
        return fail(HLBM_EINVAL, "nsteps must be in [0, %lld] (steps recorded on the tape)", R0);
    const size_t n = c->p.N;
    const size_t rows = porosity_rows(&c->cfg);  // rows of the gradient: 1 scalar, 6 tensor
    const double* gr = dJ_drho;
    const double* gu = dJ_du;
    double* gd = dJ_dd;
    void* tmp = nullptr;
    hipError_t e = hipSuccess;
    if (!on_device) {
        e = hipMalloc(&tmp, (4 + rows) * n * sizeof(double));
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        double* t = static_cast<double*>(tmp);
        e = hipMemcpyAsync(t, dJ_drho, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(t + n, dJ_du, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t + 4 * n, dJ_dd, rows * n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        gr = t;
        gu = t + n;
        gd = t + 4 * n;
    }
    const int K = c->tape_every;
    const int q = c->q, storage = c->cfg.storage, bc = c->bcmode, pk = c->cfg.porosity_kind;
    const size_t rec_step = record_step_bytes(c);  // bytes of one step's moment record
    // Reverse steps t = R0 .. tlo + 1 linearize at the moments of forward steps t.
    const long long tlo = R0 - nsteps;
    int a = 0;
    if (e == hipSuccess && nsteps > 0 && c->tape_rec) {
        // moment record of the whole run: reverse step t reads the record of
        // forward step t (relative index t - 1); nothing is replayed
        e = hlbm::launch_adjoint_seed(q, storage, bc, c->p, c->pop[c->cur], gr, gu, c->tape_lam[a], c->bx,
                                      c->stream);
        for (long long t = R0; e == hipSuccess && t > tlo; --t) {
            e = hlbm::launch_adjoint(q, storage, bc, pk, c->p, c->tape_lam[a], c->tape_lam[a ^ 1], c->dfield, gd,
                                     c->bx, c->stream, c->tape_rec + (size_t)(t - 1) * rec_step);
            a ^= 1;
        }
    } else if (e == hipSuccess && nsteps > 0) {
        // Segment m (forward steps mK + 1 .. mK + K) is replayed from its
        // checkpoint on the replay stream into set m & 1: its sweeps alternate
        // between the set's two state buffers and write the moments of each
        // step (record j = step mK + j + 1), up to the highest step a reverse
        // step of this call needs; after the reverse steps that last read
        // that set.
        auto seg_state = [&](int k, long long j) -> char* {
            return c->tape_seg + (size_t)(2 * k + (int)(j & 1)) * c->pop_bytes;
        };
        auto seg_rec = [&](int k, long long j) -> char* {
            return c->tape_segrec + ((size_t)k * (size_t)K + (size_t)j) * rec_step;
        };
        auto thi_of = [&](long long m) { return (R0 < m * K + K) ? R0 : m * K + K; };
        auto replay = [&](long long m) -> hipError_t {
            const int k = (int)(m & 1);
            // a segment the forward steps kept needs no replay (its record
            // holds steps mK + 1 .. min(R0, mK + K), all that this call reads)
            if (c->tape_kept[k] && m == kept_segment(c, k)) return hipEventRecord(c->replayed[k], c->stream);
            c->tape_kept[k] = false;  // the replay overwrites the kept record
            hipError_t r = hipStreamWaitEvent(c->tape_stream, c->consumed[k], 0);
            const long long jn = thi_of(m) - m * K;
            for (long long j = 0; j < jn && r == hipSuccess; ++j) {
                const char* src = j == 0 ? c->tape_cps + (size_t)m * c->pop_bytes : seg_state(k, j - 1);
                r = hlbm::launch_sweep(q, storage, bc, pk, c->p, src, seg_state(k, j), c->dfield, c->bx,
                                       c->tape_stream, nullptr, seg_rec(k, j));
            }
            if (r == hipSuccess) r = hipEventRecord(c->replayed[k], c->tape_stream);
            return r;
        };
        e = hlbm::launch_adjoint_seed(q, storage, bc, c->p, c->pop[c->cur], gr, gu, c->tape_lam[a], c->bx,
                                      c->stream);
        // both replay sets free, and the replay stream ordered after all work
        // queued so far (the forward steps that wrote the checkpoints)
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventRecord(c->consumed[k], c->stream);
        const long long mhi = (R0 - 1) / K, mlo = tlo / K;
        if (e == hipSuccess) e = replay(mhi);
        for (long long m = mhi; e == hipSuccess && m >= mlo; --m) {
            // the segment below replays while this one's reverse steps run
            if (m - 1 >= mlo) e = replay(m - 1);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->replayed[m & 1], 0);
            const long long thi = thi_of(m);
            const long long tmin = (tlo + 1 > m * K + 1) ? tlo + 1 : m * K + 1;
            for (long long t = thi; e == hipSuccess && t >= tmin; --t) {
                e = hlbm::launch_adjoint(q, storage, bc, pk, c->p, c->tape_lam[a], c->tape_lam[a ^ 1], c->dfield,
                                         gd, c->bx, c->stream, seg_rec((int)(m & 1), t - 1 - m * K));
                a ^= 1;
            }
            if (e == hipSuccess) e = hipEventRecord(c->consumed[m & 1], c->stream);
        }
    }
    if (e == hipSuccess && tmp)
        e = hipMemcpyAsync(dJ_dd, gd, rows * n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    // after a failed launch the replay stream may still hold queued replays
    const hipError_t e2 = hipStreamSynchronize(c->tape_stream);
    if (e == hipSuccess) e = e2;
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "adjoint");
    return HLBM_OK;
}

int hlbm_sync(hlbm_ctx* c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    if (c->batch) return batch_check_barrier(c);
    return HLBM_OK;
}

int hlbm_create_batch(const hlbm_config* items, int n_items, hlbm_ctx** out)
{
    if (!out) return fail(HLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!items) return fail(HLBM_EINVAL, "items is NULL");
    if (n_items < 1 || n_items > 65536) return fail(HLBM_EINVAL, "n_items must be in [1, 65536]");
    const int storage = items[0].storage;
    // items[0].block_x is the tile: cells per tile = threads per block
    const int tile = items[0].block_x ? items[0].block_x : hlbm::TILE_DEFAULT;
    if (tile > hlbm::TILE_MAX) return fail(HLBM_EINVAL, "a batch tile (items[0].block_x) must be <= %d", hlbm::TILE_MAX);
    unsigned long long ntot = 0, ntiles = 0, max_cells = 0;
    for (int k = 0; k < n_items; ++k) {
        const hlbm_config* it = &items[k];
        int rc = validate_config(it);
        if (rc) return fail(rc, "item %d: %s", k, hlbm_last_error());
        if (it->lattice != HLBM_D3Q19) return fail(HLBM_EUNSUPPORTED, "item %d: batches use D3Q19", k);
        if (it->porosity_kind != HLBM_POROSITY_SCALAR)
            return fail(HLBM_EUNSUPPORTED, "item %d: batch items take a scalar porosity control", k);
        if (it->storage != storage) return fail(HLBM_EINVAL, "item %d: all items share one storage", k);
        if (it->pattern != HLBM_AB) return fail(HLBM_EUNSUPPORTED, "item %d: batch items use HLBM_AB", k);
        if (k > 0 && it->row_pad_bytes != 0)
            return fail(HLBM_EINVAL, "item %d: items[0].row_pad_bytes pads the packed rows; the others must be 0", k);
        for (int a = 0; a < 3; ++a)
            if (it->bc_lo[a] != HLBM_PERIODIC || it->bc_hi[a] != HLBM_PERIODIC)
                return fail(HLBM_EUNSUPPORTED, "item %d: batch items are fully periodic", k);
        if (it->nx < 2 || it->ny < 2 || it->nz < 2 || it->nx > 1024 || it->ny > 1024 || it->nz > 1024)
            return fail(HLBM_EINVAL, "item %d: each edge must be in [2, 1024]", k);
        const unsigned long long cells = (unsigned long long)it->nx * it->ny * it->nz;
        const unsigned long long mxy = it->nx > it->ny ? it->nx : it->ny;
        if (cells * mxy >= (1ull << 32))
            return fail(HLBM_EUNSUPPORTED, "item %d: nx*ny*nz*max(nx,ny) must be < 2^32", k);
        ntot += cells;
        ntiles += (cells + tile - 1) / tile;
        if (cells > max_cells) max_cells = cells;
    }
    if (items[0].external_memory) return fail(HLBM_EUNSUPPORTED, "a batch allocates its own memory");
    if (ntot * elem_bytes(storage) >= (1ull << 32))
        return fail(HLBM_EUNSUPPORTED, "packed cells x element size must be < 4 GiB");
    hlbm_ctx* c = new (std::nothrow) hlbm_ctx();
    if (!c) return fail(HLBM_ENOMEM, "host allocation of the context failed");
    c->cfg = items[0];
    c->batch = true;
    c->n_items = n_items;
    c->batch_mode = HLBM_BATCH_GRAPH;
    c->q = 19;
    c->bcmode = hlbm::BC_PERIODIC;
    fill_params(&items[0], &c->p);
    c->p.nx = (int)ntot;
    c->p.ny = 1;
    c->p.nz = 1;
    c->p.N = (uint32_t)ntot;
    // items[0].row_pad_bytes pads the packed population rows (validated above)
    c->p.P = hlbm::row_pitch((uint32_t)ntot, elem_bytes(storage), items[0].row_pad_bytes);
    c->bx = 256;
    c->elem = elem_bytes(storage);
    c->delem = porosity_elem_bytes(storage);
    c->pop_bytes = (size_t)c->p.P * 19 * c->elem;
    c->state_bytes = (size_t)ntot * 19 * c->elem;
    c->stream = static_cast<hipStream_t>(items[0].hip_stream);
    c->own_mem = true;
    c->gsteps[0] = c->gsteps[1] = -1;
    c->items.resize(n_items);
    c->item_porosity.assign(n_items, 0);
    c->item_masked.assign(n_items, 0);
    c->n_masked = 0;
    std::vector<uint32_t> tile_item((size_t)ntiles);
    uint32_t base = 0, tile0 = 0;
    for (int k = 0; k < n_items; ++k) {
        const hlbm_config* it = &items[k];
        hlbm::BatchItem& b = c->items[k];
        b.base = base;
        b.nx = it->nx;
        b.ny = it->ny;
        b.nz = it->nz;
        b.cells = (uint32_t)it->nx * it->ny * it->nz;
        b.tile0 = tile0;
        b.mx = (uint32_t)(((1ull << 32) + it->nx - 1) / it->nx);
        b.my = (uint32_t)(((1ull << 32) + it->ny - 1) / it->ny);
        b.omega = 1.0 / it->tau;
        b.pref = 1.0 - 0.5 / it->tau;
        for (int a = 0; a < 3; ++a) b.F[a] = it->force[a];
        const uint32_t nt = (b.cells + tile - 1) / tile;
        for (uint32_t j = 0; j < nt; ++j) tile_item[tile0 + j] = (uint32_t)k;
        base += b.cells;
        tile0 += nt;
    }
    hipError_t e = hipMalloc(&c->pop[0], c->pop_bytes);
    if (e == hipSuccess) e = hipMalloc(&c->pop[1], c->pop_bytes);
    if (e == hipSuccess) e = hipMalloc(&c->dfield, (size_t)ntot * c->delem);
    if (e == hipSuccess) e = hipMalloc(&c->items_dev, sizeof(hlbm::BatchItem) * n_items);
    if (e == hipSuccess) e = hipMalloc(&c->tile_item_dev, sizeof(uint32_t) * (size_t)ntiles);
    if (e == hipSuccess) e = hipMalloc(&c->tile_partials, sizeof(double) * 4 * (size_t)ntiles);
    if (e == hipSuccess) e = hipMalloc(&c->item_totals_dev, sizeof(double) * 4 * (size_t)n_items);
    if (e == hipSuccess) e = hipMalloc(&c->bar_sync, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&c->bar_err, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->flag_out, sizeof(int));
    if (e != hipSuccess) {
        hlbm_destroy(c);
        return fail(HLBM_ENOMEM, "device allocation for the batch failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(c->items_dev, c->items.data(), sizeof(hlbm::BatchItem) * n_items, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->tile_item_dev, tile_item.data(), sizeof(uint32_t) * (size_t)ntiles, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->bar_err, 0, sizeof(int));
    int per_cu = 0, cus = 0;
    if (e == hipSuccess) e = hlbm::batch_occupancy(storage, tile, &per_cu);
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        hlbm_destroy(c);
        return hip_fail(e, "batch set-up");
    }
    if (per_cu < 1) {
        hlbm_destroy(c);
        return fail(HLBM_EUNSUPPORTED, "no block of %d threads of the batched kernel fits on a CU", tile);
    }
    c->cus = cus;
    c->max_blocks_per_cu = per_cu;
    c->bl.items = c->items_dev;
    c->bl.tile_item = c->tile_item_dev;
    c->bl.n_items = (uint32_t)n_items;
    c->bl.ntiles = (uint32_t)ntiles;
    c->bl.Ntot = c->p.P;  // row stride of the packed populations
    c->bl.rho0 = c->p.rho0;
    c->bl.scale = c->p.scale;
    c->bl.sync = c->bar_sync;
    c->bl.err = c->bar_err;
    c->bl.spin_limit = kBarrierPollsDefault;
    c->bl.tile = (uint32_t)tile;
    set_batch_schedule(c, 0, 0);
    c->bound = true;
    int rc = zero_state(c);
    if (rc) {
        hlbm_destroy(c);
        return rc;
    }
    *out = c;
    return HLBM_OK;
}

int hlbm_batch_info(const hlbm_ctx* c, int* n_items, size_t* total_cells)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (n_items) *n_items = c->n_items;
    if (total_cells) *total_cells = c->p.N;
    return HLBM_OK;
}

int hlbm_batch_set_mode(hlbm_ctx* c, int mode)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (mode < HLBM_BATCH_GRAPH || mode > HLBM_BATCH_GRAPH_PERSISTENT)
        return fail(HLBM_EINVAL, "unknown batch mode %d", mode);
    c->batch_mode = mode;
    return HLBM_OK;
}

int hlbm_batch_set_schedule(hlbm_ctx* c, int blocks_per_cu, int chunk)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (blocks_per_cu < 0 || blocks_per_cu > c->max_blocks_per_cu)
        return fail(HLBM_EINVAL, "blocks_per_cu must be in [0, %d] for tiles of %u cells", c->max_blocks_per_cu,
                    c->bl.tile);
    if (chunk < 0 || chunk > hlbm::CHUNK_MAX) return fail(HLBM_EINVAL, "chunk must be in [0, %d]", hlbm::CHUNK_MAX);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "batch_set_schedule: outstanding work failed");
    set_batch_schedule(c, blocks_per_cu, chunk);
    return HLBM_OK;
}

int hlbm_batch_set_barrier_limit(hlbm_ctx* c, int polls)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (polls < 0) return fail(HLBM_EINVAL, "polls must be >= 0");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "batch_set_barrier_limit: outstanding work failed");
    c->bl.spin_limit = (unsigned)polls;
    for (int k = 0; k < 2; ++k) {  // the graphs hold the old bound
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
        c->gsteps[k] = -1;
    }
    return HLBM_OK;
}

int hlbm_batch_get_schedule(const hlbm_ctx* c, int* tile, int* blocks_per_cu, int* max_blocks_per_cu, int* chunk)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (tile) *tile = (int)c->bl.tile;
    if (blocks_per_cu) *blocks_per_cu = c->batch_bpc;
    if (max_blocks_per_cu) *max_blocks_per_cu = c->max_blocks_per_cu;
    if (chunk) *chunk = (int)c->bl.chunk;
    return HLBM_OK;
}

int hlbm_batch_set_porosity(hlbm_ctx* c, int item, const void* d, int dtype, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (item < 0 || item >= c->n_items) return fail(HLBM_EINVAL, "item %d out of range", item);
    if (!d) return fail(HLBM_EINVAL, "porosity array is NULL");
    if (dtype < HLBM_DT_F64 || dtype > HLBM_DT_F16) return fail(HLBM_EINVAL, "unknown dtype %d", dtype);
    const hlbm::BatchItem& it = c->items[item];
    const size_t in_elem = dtype == HLBM_DT_F64 ? 8 : (dtype == HLBM_DT_F32 ? 4 : 2);
    const size_t n = it.cells;
    const void* src = d;
    void* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
        e = hipMalloc(&tmp, n * in_elem);
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        e = hipMemcpyAsync(tmp, d, n * in_elem, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return hip_fail(e, "porosity upload");
        }
        src = tmp;
    }
    void* out = static_cast<char*>(c->dfield) + (size_t)it.base * c->delem;
    e = hlbm::launch_porosity_convert(dtype, src, c->cfg.storage, hlbm::PK_SCALAR, out, (uint32_t)n, (uint32_t)n, c->flag_out,
                                      c->stream);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, c->flag_out, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "porosity conversion");
    if (flag) {
        c->item_porosity[item] = 0;
        c->porosity_set = false;
        return fail(HLBM_EINVAL, "item %d: porosity values must be finite and in [0, 1]", item);
    }
    c->item_porosity[item] = 1;
    bool all = true;
    for (int k = 0; k < c->n_items; ++k) all = all && c->item_porosity[k];
    c->porosity_set = all;
    return HLBM_OK;
}

int hlbm_batch_set_solid_mask(hlbm_ctx* c, int item, const unsigned char* mask, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    if (item < 0 || item >= c->n_items) return fail(HLBM_EINVAL, "item %d out of range", item);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "batch_set_solid_mask: outstanding work failed");
    const hlbm::BatchItem& it = c->items[item];
    const size_t ntot = c->p.N;
    if (!mask && !c->item_masked[item]) return HLBM_OK;
    if (!c->linkmask) {
        // zero link masks: items without obstacles load what the periodic gather loads
        e = hipMalloc(&c->linkmask, ntot * sizeof(uint32_t));
        if (e != hipSuccess) {
            c->linkmask = nullptr;
            return fail(HLBM_ENOMEM, "link mask allocation: %s", hipGetErrorString(e));
        }
        e = hipMemsetAsync(c->linkmask, 0, ntot * sizeof(uint32_t), c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "clearing the link mask");
    }
    uint32_t* rows = c->linkmask + it.base;
    if (!mask) {
        e = hipMemsetAsync(rows, 0, (size_t)it.cells * sizeof(uint32_t), c->stream);
    } else {
        const unsigned char* src = mask;
        void* tmp = nullptr;
        if (!on_device) {
            e = hipMalloc(&tmp, it.cells);
            if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
            e = hipMemcpyAsync(tmp, mask, it.cells, hipMemcpyHostToDevice, c->stream);
            src = static_cast<const unsigned char*>(tmp);
        }
        hlbm::Params ip = c->p;
        ip.nx = (int)it.nx;
        ip.ny = (int)it.ny;
        ip.nz = (int)it.nz;
        ip.N = it.cells;
        if (e == hipSuccess) e = hlbm::launch_linkmask(19, ip, src, rows, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (tmp) (void)hipFree(tmp);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "batch solid mask");
    c->n_masked += (mask ? 1 : 0) - (c->item_masked[item] ? 1 : 0);
    c->item_masked[item] = mask ? 1 : 0;
    // the masked kernels run while any item holds obstacles; the graphs hold
    // the old kernels
    c->bl.linkmask = c->n_masked ? c->linkmask : nullptr;
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
        c->gsteps[k] = -1;
    }
    return HLBM_OK;
}

int hlbm_batch_moments(hlbm_ctx* c, int item, double* drho, double* u, int on_device, double* totals)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->batch) return fail(HLBM_EINVAL, "not a batch context");
    const bool fields = drho || u;
    if (fields && (item < 0 || item >= c->n_items)) return fail(HLBM_EINVAL, "item %d out of range", item);
    if (fields && (!drho || !u)) return fail(HLBM_EINVAL, "give both drho and u, or neither");
    const size_t n = fields ? c->items[item].cells : 0;
    double* ddr = drho;
    double* du = u;
    void* tmp = nullptr;
    hipError_t e;
    if (fields && !on_device) {
        e = hipMalloc(&tmp, 4 * n * sizeof(double));
        if (e != hipSuccess) return fail(HLBM_ENOMEM, "staging allocation: %s", hipGetErrorString(e));
        ddr = static_cast<double*>(tmp);
        du = ddr + n;
    }
    e = hlbm::launch_batch_moments(c->cfg.storage, c->bl, c->pop[c->cur], c->tile_partials,
                                   fields ? item : -1, fields ? ddr : nullptr, fields ? du : nullptr,
                                   c->item_totals_dev, c->stream);
    if (e == hipSuccess && totals)
        e = hipMemcpyAsync(totals, c->item_totals_dev, 4 * sizeof(double) * c->n_items,
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && tmp) e = hipMemcpyAsync(drho, ddr, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && tmp) e = hipMemcpyAsync(u, du, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "batch moments");
    rc = batch_check_barrier(c);
    if (rc) return rc;
    if (totals)
        for (int k = 0; k < 4 * c->n_items; ++k)
            if (!isfinite(totals[k])) return fail(HLBM_ENUMERIC, "non-finite total (item %d)", k / 4);
    return HLBM_OK;
}

}  // extern "C"
