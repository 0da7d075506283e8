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

#include <new>

#include "hlbm.h"
#include "hlbm_internal.hpp"
#include "lattice.hpp"

using hlbm::Params;

struct hlbm_ctx {
    hlbm_config cfg;
    Params p;
    int q;
    int bcmode;
    int bx;
    size_t elem;       // bytes per stored population value
    size_t delem;      // bytes per porosity value
    size_t pop_bytes;  // one population buffer
    void* pop[2];
    void* dfield;
    bool own_mem;
    bool bound;
    bool porosity_set;
    int cur;           // buffer holding the current post-collision state
    long long step;
    hipStream_t stream;
    double* partials;  // FP64 per-block partials for the totals
    uint32_t partials_blocks;
    double* totals_dev;
    int* flags_dev;    // per-block flags of the porosity check
    uint32_t flags_blocks;
    int* flag_out;
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

int validate_config(const hlbm_config* c)
{
    if (!c) return fail(HLBM_EINVAL, "config is NULL");
    if (c->lattice != HLBM_D2Q9 && c->lattice != HLBM_D3Q19)
        return fail(HLBM_EINVAL, "lattice must be HLBM_D2Q9 or HLBM_D3Q19 (got %d)", c->lattice);
    if (elem_bytes(c->storage) == 0) return fail(HLBM_EINVAL, "unknown storage %d", c->storage);
    if (c->pattern != HLBM_AB) return fail(HLBM_EUNSUPPORTED, "pattern %d not provided", c->pattern);
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
    return HLBM_OK;
}

void fill_params(const hlbm_config* c, Params* p)
{
    memset(p, 0, sizeof(*p));
    p->nx = c->nx;
    p->ny = c->ny;
    p->nz = c->nz;
    p->N = (uint32_t)((unsigned long long)c->nx * c->ny * c->nz);
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
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMemsetAsync(c->pop[k], 0, c->pop_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(e, "zeroing populations");
    }
    c->cur = 0;
    c->step = 0;
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
    if (pop_bytes) *pop_bytes = n * (size_t)cfg->lattice * elem_bytes(cfg->storage);
    if (porosity_bytes) *porosity_bytes = n * porosity_elem_bytes(cfg->storage);
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
    bool general = false;
    for (int a = 0; a < 3; ++a)
        if (cfg->bc_lo[a] != HLBM_PERIODIC) general = true;
    c->bcmode = general ? hlbm::BC_GENERAL : hlbm::BC_PERIODIC;
    c->bx = cfg->block_x ? cfg->block_x : auto_block_x(cfg->nx);
    c->elem = elem_bytes(cfg->storage);
    c->delem = porosity_elem_bytes(cfg->storage);
    c->pop_bytes = (size_t)c->p.N * (size_t)c->q * c->elem;
    c->stream = static_cast<hipStream_t>(cfg->hip_stream);
    c->own_mem = !cfg->external_memory;
    if (c->own_mem) {
        hipError_t e = hipMalloc(&c->pop[0], c->pop_bytes);
        if (e == hipSuccess) e = hipMalloc(&c->pop[1], c->pop_bytes);
        if (e == hipSuccess) e = hipMalloc(&c->dfield, (size_t)c->p.N * c->delem);
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
    const uint32_t nfl = (c->p.N + 255) / 256;
    hipError_t e = hipMalloc(&c->flags_dev, sizeof(int) * (size_t)nfl);
    if (e == hipSuccess) e = hipMalloc(&c->flag_out, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&c->totals_dev, 4 * sizeof(double));
    if (e != hipSuccess) {
        hlbm_destroy(c);
        return fail(HLBM_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    c->flags_blocks = nfl;
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
    if (!pop_a || !pop_b || !porosity) return fail(HLBM_EINVAL, "NULL buffer");
    if (pop_a == pop_b) return fail(HLBM_EINVAL, "population buffers must differ");
    if (((uintptr_t)pop_a | (uintptr_t)pop_b | (uintptr_t)porosity) & 255u)
        return fail(HLBM_EINVAL, "buffers must be 256-byte aligned");
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->dfield = porosity;
    c->bound = true;
    c->porosity_set = false;
    return zero_state(c);
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
    if (c->flags_dev) (void)hipFree(c->flags_dev);
    if (c->flag_out) (void)hipFree(c->flag_out);
    delete c;
    return rc;
}

int hlbm_set_porosity(hlbm_ctx* c, const void* d, int dtype, int on_device)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!d) return fail(HLBM_EINVAL, "porosity array is NULL");
    if (dtype < HLBM_DT_F64 || dtype > HLBM_DT_F16) return fail(HLBM_EINVAL, "unknown dtype %d", dtype);
    const size_t in_elem = dtype == HLBM_DT_F64 ? 8 : (dtype == HLBM_DT_F32 ? 4 : 2);
    const size_t n = c->p.N;
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
    e = hlbm::launch_porosity_convert(dtype, src, c->cfg.storage, c->dfield, (uint32_t)n,
                                      c->flags_dev, c->flag_out, c->stream);
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, c->flag_out, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "porosity conversion");
    if (flag) {
        c->porosity_set = false;
        return fail(HLBM_EINVAL, "porosity values must be finite and in [0, 1]");
    }
    c->porosity_set = true;
    return HLBM_OK;
}

int hlbm_step(hlbm_ctx* c, int nsteps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(HLBM_EINVAL, "nsteps must be >= 0");
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!c->porosity_set) return fail(HLBM_ESTATE, "porosity not set");
    for (int t = 0; t < nsteps; ++t) {
        hipError_t e = hlbm::launch_sweep(c->q, c->cfg.storage, c->bcmode, c->p, c->pop[c->cur],
                                          c->pop[c->cur ^ 1], c->dfield, c->bx, c->stream);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
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
    e = hlbm::launch_moments(c->q, c->cfg.storage, c->bcmode, c->p, c->pop[c->cur], ddr, du,
                             dtype == HLBM_DT_F64, partials, c->bx, c->stream);
    if (e == hipSuccess && totals) e = hlbm::launch_reduce4(partials, l.nblocks, c->totals_dev, c->stream);
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

int hlbm_state_bytes(const hlbm_ctx* c, size_t* bytes)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!bytes) return fail(HLBM_EINVAL, "bytes is NULL");
    *bytes = c->pop_bytes;
    return HLBM_OK;
}

int hlbm_get_state(hlbm_ctx* c, void* dst, int on_device, long long* step)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    if (!dst) return fail(HLBM_EINVAL, "dst is NULL");
    hipError_t e = hipMemcpyAsync(dst, c->pop[c->cur], c->pop_bytes,
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
    hipError_t e = hipMemcpyAsync(c->pop[c->cur], src, c->pop_bytes,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "set_state");
    c->step = step;
    return HLBM_OK;
}

int hlbm_reset(hlbm_ctx* c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!c->bound) return fail(HLBM_ESTATE, "buffers not bound");
    return zero_state(c);
}

int hlbm_sync(hlbm_ctx* c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    return HLBM_OK;
}

}  // extern "C"
