// C ABI of the induced-dipole library: context, validation, and the entry points declared in
// include/amoeba.h.  Host code here only validates, allocates and sequences kernels; every
// step of the computation runs in the HIP kernels of this directory.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "common.h"
#include "reduce.h"

namespace amoeba {

int set_error(amoeba_ctx* c, int code, const std::string& msg)
{
    if (c)
        c->err = msg;
    return code;
}

int hip_check(amoeba_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess)
        return AMOEBA_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(c, e == hipErrorOutOfMemory ? AMOEBA_E_NOMEM : AMOEBA_E_DEVICE, m);
}

StageTimer::StageTimer(amoeba_ctx* ctx, int stage, hipStream_t stream) : c(ctx), st(stream ? stream : ctx->stream)
{
    if (!c->timing && !(c->timing_live && stage == AMOEBA_T_REAL))
        return;
    size_t need = c->trec.size() * 2 + 2;
    while (c->tev.size() < need) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return;
        c->tev.push_back(e);
    }
    idx = (int)c->trec.size() * 2;
    c->trec.push_back({stage, idx});
    hipEventRecord(c->tev[idx], st);
}

StageTimer::~StageTimer()
{
    if (idx >= 0)
        hipEventRecord(c->tev[idx + 1], st);
}

int ctx_alloc(amoeba_ctx* c, void** p, size_t bytes)
{
    if (bytes == 0)
        bytes = 16;
    // the stored pair coefficients are optional: they give way to any other allocation
    if (c->prm.max_workspace_bytes > 0 && c->ws_bytes + (int64_t)bytes > c->prm.max_workspace_bytes && c->coef)
        coef_release(c);
    if (c->prm.max_workspace_bytes > 0 && c->ws_bytes + (int64_t)bytes > c->prm.max_workspace_bytes)
        return set_error(c, AMOEBA_E_NOMEM, "device workspace would exceed max_workspace_bytes (" +
                                                std::to_string(c->ws_bytes + (int64_t)bytes) + " > " +
                                                std::to_string(c->prm.max_workspace_bytes) + ")");
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess)
        return set_error(c, AMOEBA_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    hipMemsetAsync(q, 0, bytes, c->stream);
    c->allocs.push_back(q);
    c->ws_bytes += (int64_t)bytes;
    *p = q;
    return AMOEBA_OK;
}

// ------------------------------------------------------------------------------------------
// validation kernels
// ------------------------------------------------------------------------------------------
__global__ void k_validate_atoms(int n, const double* __restrict__ alpha, const double* __restrict__ thole,
                                 const int* __restrict__ ptr, const int* __restrict__ sj,
                                 const double* __restrict__ ss, long long nnz, int* __restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n)
        return;
    if (i == n) {
        if (ptr[0] != 0 || (long long)ptr[n] != nnz)
            atomicOr(flags, kFlagBadCsr);
        return;
    }
    double a = alpha[i], t = thole[i];
    if (!(a > 0.0) || !isfinite(a))
        atomicOr(flags, kFlagBadAlpha);
    if (!(t >= 0.0) || !isfinite(t))
        atomicOr(flags, kFlagBadThole);
    int b = ptr[i], e = ptr[i + 1];
    if (b > e || b < 0 || (long long)e > nnz) {
        atomicOr(flags, kFlagBadCsr);
        return;
    }
    for (int k = b; k < e; ++k) {
        int j = sj[k];
        double s = ss[k];
        if (j < 0 || j >= n || j == i || !isfinite(s)) {
            atomicOr(flags, kFlagBadCsr);
            return;
        }
        // the reverse entry must exist with the same scale
        int jb = ptr[j], je = ptr[j + 1];
        bool found = false;
        if (jb >= 0 && je <= nnz && jb <= je)
            for (int m = jb; m < je; ++m)
                if (sj[m] == i && ss[m] == s) {
                    found = true;
                    break;
                }
        if (!found) {
            atomicOr(flags, kFlagBadCsr);
            return;
        }
    }
}

__global__ void k_check_finite(size_t n, const double* __restrict__ v, int* __restrict__ flags)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i]))
        atomicOr(flags, kFlagNonFinite);
}

__global__ void k_check_overflow(size_t n, const double* __restrict__ v, double lim, int* __restrict__ flags)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(fabs(v[i]) < lim))
        atomicOr(flags, isfinite(v[i]) ? kFlagOverflow : kFlagNonFinite);
}

// multipoles into slot order: (q, d), (Txx, Txy, Txz, Tyy), (Tyz, Tzz, 0, 0); traceless check
__global__ void k_gather_mpole(int npad, const int* __restrict__ perm, const double* __restrict__ q,
                               const double* __restrict__ dip, const double* __restrict__ quad,
                               double4* __restrict__ md, float4* __restrict__ mf, int* __restrict__ flags)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (a >= 0) {
        v[0] = q[a];
        for (int c = 0; c < 3; ++c)
            v[1 + c] = dip[3 * (size_t)a + c];
        for (int c = 0; c < 6; ++c)
            v[4 + c] = quad[6 * (size_t)a + c];
        for (int c = 0; c < 10; ++c)
            if (!isfinite(v[c]))
                atomicOr(flags, kFlagNonFinite);
        double tr = v[4] + v[7] + v[9];
        double sc = fabs(v[4]) + fabs(v[7]) + fabs(v[9]);
        if (fabs(tr) > 1e-10 * (1.0 + sc))
            atomicOr(flags, kFlagBadCsr);  // reported as "quadrupole not traceless"
    }
    md[3 * (size_t)s] = make_double4(v[0], v[1], v[2], v[3]);
    md[3 * (size_t)s + 1] = make_double4(v[4], v[5], v[6], v[7]);
    md[3 * (size_t)s + 2] = make_double4(v[8], v[9], 0.0, 0.0);
    if (mf) {
        mf[3 * (size_t)s] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
        mf[3 * (size_t)s + 1] = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
        mf[3 * (size_t)s + 2] = make_float4((float)v[8], (float)v[9], 0.f, 0.f);
    }
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

int sort_params(amoeba_ctx* c);

int read_flags(amoeba_ctx* c, int* out)
{
    hipMemcpyAsync(c->flags_host, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "flags");
    *out = c->flags_host[0];
    return rc;
}

int check_vec_finite(amoeba_ctx* c, const double* v, size_t n, const char* what)
{
    hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
    hipLaunchKernelGGL(k_check_finite, dim3(nblk(n, 256)), dim3(256), 0, c->stream, n, v, c->flags);
    int f = 0, rc = read_flags(c, &f);
    if (rc)
        return rc;
    if (f & kFlagNonFinite)
        return set_error(c, AMOEBA_E_NUMERIC, std::string("non-finite value in ") + what);
    return AMOEBA_OK;
}

static int ready(amoeba_ctx* c, const char* who)
{
    if (!c->atoms_set)
        return set_error(c, AMOEBA_E_STATE, std::string(who) + ": amoeba_set_atoms has not been called");
    if (!c->list_built)
        return set_error(c, AMOEBA_E_LIST, std::string(who) + ": amoeba_build_blocklist has not been called");
    return AMOEBA_OK;
}

// Queue the range check of a slot-order field (read with the caller's next flags read).
void launch_check_overflow(amoeba_ctx* c, const double* v_slot)
{
    const size_t n3 = 3 * (size_t)c->npad;
    hipLaunchKernelGGL(k_check_overflow, dim3(nblk(n3, 256)), dim3(256), 0, c->stream, n3, v_slot, kFixRange,
                       c->flags);
}

static int check_overflow(amoeba_ctx* c, const double* v_slot)
{
    if (!c->mixed)
        return AMOEBA_OK;
    size_t n3 = 3 * (size_t)c->npad;
    hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
    hipLaunchKernelGGL(k_check_overflow, dim3(nblk(n3, 256)), dim3(256), 0, c->stream, n3, v_slot, kFixRange,
                       c->flags);
    int f = 0, rc = read_flags(c, &f);
    if (rc)
        return rc;
    if (f & kFlagNonFinite)
        return set_error(c, AMOEBA_E_NUMERIC, "non-finite field");
    if (f & kFlagOverflow)
        return set_error(c, AMOEBA_E_OVERFLOW, "field outside the exact fixed-point range (|E| >= 8192 e/A^2)");
    return AMOEBA_OK;
}

int begin_config(amoeba_ctx* c, const double* pos, const char* who)
{
    int rc = ready(c, who);
    if (rc)
        return rc;
    if (!pos)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": NULL pos");
    return prepare_config(c, pos);
}

}  // namespace amoeba

using namespace amoeba;

static thread_local std::string g_create_error;

extern "C" {

const char* amoeba_create_error(void) { return g_create_error.c_str(); }

int amoeba_create(const amoeba_params* p, void* hip_stream, amoeba_ctx** out)
{
    g_create_error.clear();
    auto bad = [](int code, const std::string& m) {
        g_create_error = m;
        return code;
    };
    if (!p || !out)
        return bad(AMOEBA_E_INVALID, "amoeba_create: NULL params or out");
    *out = nullptr;
    if (p->n_atoms < 1 || p->n_atoms > (1 << 26))
        return bad(AMOEBA_E_INVALID, "n_atoms must be in [1, 2^26]");
    double bmin = 1e300;
    for (int a = 0; a < 3; ++a) {
        if (!(p->box[a] > 0.0) || !std::isfinite(p->box[a]))
            return bad(AMOEBA_E_INVALID, "box edges must be positive and finite");
        bmin = std::fmin(bmin, p->box[a]);
    }
    if (!(p->cutoff > 0.0) || !std::isfinite(p->cutoff))
        return bad(AMOEBA_E_INVALID, "cutoff must be positive");
    if (!(p->buffer >= 0.0) || !std::isfinite(p->buffer))
        return bad(AMOEBA_E_INVALID, "buffer must be >= 0");
    if (!(p->cutoff + p->buffer < 0.5 * bmin))
        return bad(AMOEBA_E_INVALID, "cutoff + buffer must be smaller than half the smallest box edge");
    if (!(p->ewald_alpha > 0.0) || !std::isfinite(p->ewald_alpha))
        return bad(AMOEBA_E_INVALID, "ewald_alpha must be positive");
    if (p->order != 5)
        return bad(AMOEBA_E_INVALID, "only B-spline order 5 is supported");
    for (int a = 0; a < 3; ++a)
        if (p->grid[a] < 2 * p->order || p->grid[a] > 2048)
            return bad(AMOEBA_E_INVALID, "grid sizes must be in [2*order, 2048]");
    if (p->precision != AMOEBA_FP64 && p->precision != AMOEBA_MIXED)
        return bad(AMOEBA_E_INVALID, "precision must be AMOEBA_FP64 or AMOEBA_MIXED");
    if (p->max_workspace_bytes < 0)
        return bad(AMOEBA_E_INVALID, "max_workspace_bytes must be >= 0");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return bad(AMOEBA_E_DEVICE, "no HIP device available");
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return bad(AMOEBA_E_DEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return bad(AMOEBA_E_DEVICE, std::string("this library is built for gfx950; device is ") + prop.gcnArchName);

    amoeba_ctx* c = new amoeba_ctx();
    c->prm = *p;
    c->stream = (hipStream_t)hip_stream;
    c->device = dev;
    c->n = p->n_atoms;
    c->nb = (c->n + kBlock - 1) / kBlock;
    c->npad = c->nb * kBlock;
    c->mixed = p->precision == AMOEBA_MIXED;
    int rc = AMOEBA_OK;
    size_t np = c->npad, n3 = 3 * np;
    // partials of the grid reductions: up to one per 256-thread workgroup over 3 npad threads
    // (vector kernels) or one per PME brick, 4 values each
    size_t nbricks = 1;
    for (int a = 0; a < 3; ++a)
        nbricks *= (size_t)((p->grid[a] + kBrick - 1) / kBrick);
    size_t part_n = (std::max((size_t)nblk(3 * np, 256), nbricks) + (size_t)kRedBlocks) * 4;
    do {
        if ((rc = ctx_alloc(c, (void**)&c->perm, sizeof(int) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->slot, sizeof(int) * c->n)) ||
            (rc = ctx_alloc(c, (void**)&c->par_d, sizeof(double4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->alpha_s, sizeof(double) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->alpha_inv_s, sizeof(double) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->par_f, sizeof(float4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->sc_ptr, sizeof(int) * (np + 1))) ||
            (rc = ctx_alloc(c, (void**)&c->sc_ptr_in, sizeof(int) * (c->n + 1))) ||
            (rc = ctx_alloc(c, (void**)&c->alpha_in, sizeof(double) * c->n)) ||
            (rc = ctx_alloc(c, (void**)&c->thole_in, sizeof(double) * c->n)) ||
            (rc = ctx_alloc(c, (void**)&c->pos_s, sizeof(double4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->pos_ref, sizeof(double4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->blk_org, sizeof(double4) * c->nb)) ||
            (rc = ctx_alloc(c, (void**)&c->off_d, sizeof(double4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->off_f, sizeof(float4) * np)) ||
            (rc = ctx_alloc(c, (void**)&c->blk_tile0, sizeof(int) * (c->nb + 1))) ||
            (rc = ctx_alloc(c, (void**)&c->erec, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->v_mu, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->v_r, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->v_p, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->v_q, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->v_e, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->sc, sizeof(PcgScalars))) ||
            (rc = ctx_alloc(c, (void**)&c->red.part, sizeof(double) * part_n)) ||
            (rc = ctx_alloc(c, (void**)&c->flags, sizeof(int) * 256)) ||
            (rc = ctx_alloc(c, (void**)&c->b_cnt, sizeof(int) * (np + 1))) ||
            (rc = ctx_alloc(c, (void**)&c->b_scan, sizeof(int) * 2 * (np / 1024 + 2))))
            break;
        c->b_extent = (double*)(c->flags + 4);  // read back with the flags after a list build
        if ((rc = ctx_alloc(c, (void**)&c->eipart, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->ereal, sizeof(double) * n3)) ||
            (rc = ctx_alloc(c, (void**)&c->rev_ptr, sizeof(int) * (np + 1))))
            break;
        if (c->mixed) {
            if ((rc = ctx_alloc(c, (void**)&c->pv_f, sizeof(float4) * np)))
                break;
        } else {
            if ((rc = ctx_alloc(c, (void**)&c->pv_d, sizeof(double4) * np)))
                break;
        }
        if (hipHostMalloc((void**)&c->sc_host, sizeof(PcgScalars) * 2, hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer((void**)&c->sc_host_dev, c->sc_host, 0) != hipSuccess ||
            hipHostMalloc((void**)&c->flags_host, 64, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&c->pairs_host, 64, hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer((void**)&c->pairs_host_dev, c->pairs_host, 0) != hipSuccess) {
            rc = set_error(c, AMOEBA_E_NOMEM, "pinned host allocation failed");
            break;
        }
        if (hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_pairs, hipEventDisableTiming) != hipSuccess ||
            hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
            rc = set_error(c, AMOEBA_E_DEVICE, "hipEventCreate failed");
            break;
        }
        if ((rc = pme_setup(c)) || (rc = guess_scratch_init(c)))
            break;
        rc = hip_check(c, hipStreamSynchronize(c->stream), "amoeba_create");
    } while (false);
    if (rc != AMOEBA_OK) {
        g_create_error = c->err;
        amoeba_destroy(c);
        return rc;
    }
    *out = c;
    return AMOEBA_OK;
}

int amoeba_destroy(amoeba_ctx* c)
{
    if (!c)
        return AMOEBA_OK;
    hipStreamSynchronize(c->stream);
    if (c->stream2) {
        hipStreamSynchronize(c->stream2);
        hipStreamDestroy(c->stream2);
    }
    iteration_graph_release(c);
    if (c->gstream)
        hipStreamDestroy(c->gstream);
    for (void* p : c->allocs)
        hipFree(p);
    if (c->sc_host)
        hipHostFree(c->sc_host);
    if (c->plan_fwd)
        rocfft_plan_destroy(c->plan_fwd);
    if (c->plan_bwd)
        rocfft_plan_destroy(c->plan_bwd);
    if (c->exec_fwd)
        rocfft_execution_info_destroy(c->exec_fwd);
    if (c->exec_bwd)
        rocfft_execution_info_destroy(c->exec_bwd);
    if (c->flags_host)
        hipHostFree(c->flags_host);
    if (c->pairs_host)
        hipHostFree(c->pairs_host);
    coef_release(c);
    if (c->g_scal_host)
        hipHostFree(c->g_scal_host);
    for (auto& e : c->ev)
        if (e)
            hipEventDestroy(e);
    if (c->ev_fork)
        hipEventDestroy(c->ev_fork);
    if (c->ev_join)
        hipEventDestroy(c->ev_join);
    if (c->ev_pairs)
        hipEventDestroy(c->ev_pairs);
    for (auto& e : c->tev)
        hipEventDestroy(e);
    delete c;
    return AMOEBA_OK;
}

const char* amoeba_last_error(const amoeba_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int amoeba_set_atoms(amoeba_ctx* c, const double* alpha, const double* thole, const int32_t* sc_ptr,
                     const int32_t* sc_j, const double* sc_s, int64_t n_scaled)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!alpha || !thole || !sc_ptr)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_atoms: NULL alpha, thole or sc_ptr");
    if (n_scaled < 0 || n_scaled > (int64_t)1 << 31)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_atoms: n_scaled out of range");
    if (n_scaled > 0 && (!sc_j || !sc_s))
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_atoms: NULL sc_j or sc_s with n_scaled > 0");
    hipStream_t st = c->stream;
    int rc;
    if (n_scaled > c->n_scaled || !c->sc_j_in) {
        size_t cap = (size_t)std::max<int64_t>(n_scaled, 1);
        if ((rc = ctx_alloc(c, (void**)&c->sc_j_in, sizeof(int) * cap)) ||
            (rc = ctx_alloc(c, (void**)&c->sc_s_in, sizeof(double) * cap)) ||
            (rc = ctx_alloc(c, (void**)&c->sc_j, sizeof(int) * cap)) ||
            (rc = ctx_alloc(c, (void**)&c->sc_s, sizeof(double) * cap)))
            return rc;
    }
    hipMemsetAsync(c->flags, 0, sizeof(int), st);
    hipLaunchKernelGGL(k_validate_atoms, dim3(nblk(c->n + 1, 256)), dim3(256), 0, st, c->n, alpha, thole, sc_ptr,
                       n_scaled ? sc_j : c->sc_j_in, n_scaled ? sc_s : c->sc_s_in, (long long)n_scaled, c->flags);
    int f = 0;
    if ((rc = read_flags(c, &f)))
        return rc;
    if (f & kFlagBadAlpha)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_atoms: polarizabilities must be positive and finite");
    if (f & kFlagBadThole)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_atoms: Thole parameters must be >= 0 and finite");
    if (f & kFlagBadCsr)
        return set_error(c, AMOEBA_E_INVALID,
                         "amoeba_set_atoms: scaled-pair CSR invalid (ptr not monotone from 0 to n_scaled, "
                         "partner out of range or equal to the atom, non-finite scale, or a pair not listed "
                         "in both directions with the same scale)");
    hipMemcpyAsync(c->alpha_in, alpha, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st);
    hipMemcpyAsync(c->thole_in, thole, sizeof(double) * c->n, hipMemcpyDeviceToDevice, st);
    hipMemcpyAsync(c->sc_ptr_in, sc_ptr, sizeof(int) * (c->n + 1), hipMemcpyDeviceToDevice, st);
    if (n_scaled) {
        hipMemcpyAsync(c->sc_j_in, sc_j, sizeof(int) * n_scaled, hipMemcpyDeviceToDevice, st);
        hipMemcpyAsync(c->sc_s_in, sc_s, sizeof(double) * n_scaled, hipMemcpyDeviceToDevice, st);
    }
    c->n_scaled = n_scaled;
    c->atoms_set = true;
    c->dscales_set = false;  // direct scales belong to a pair list: set them again after this
    if (c->list_built && (rc = sort_params(c)))
        return rc;
    return hip_check(c, hipStreamSynchronize(st), "amoeba_set_atoms");
}

int amoeba_build_blocklist(amoeba_ctx* c, const double* pos)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!pos)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_build_blocklist: NULL pos");
    int rc = build_blocklist(c, pos);
    if (rc)
        c->list_built = false;
    return rc;
}

int amoeba_update_blocklist(amoeba_ctx* c, const double* pos, int32_t* rebuilt_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (rebuilt_out)
        *rebuilt_out = 0;
    if (!pos)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_update_blocklist: NULL pos");
    if (c->atoms_set && c->list_built) {
        // the displacement test of every configuration change; a stale list is rebuilt below
        int rc = begin_config(c, pos, "amoeba_update_blocklist");
        if (rc != AMOEBA_E_LIST)
            return rc;
        c->err.clear();
    }
    int rc = build_blocklist(c, pos);
    if (rc) {
        c->list_built = false;
        return rc;
    }
    if (rebuilt_out)
        *rebuilt_out = 1;
    return AMOEBA_OK;
}

// The parts of E_perm shared by the scale sets (multipoles in slot order, the unscaled tiles'
// sums in ereal, the reciprocal field in erec), leaving the flags unread.
static int perm_field_parts(amoeba_ctx* c, const double* pos, const double* q, const double* dip,
                            const double* quad, const char* what, int* flags = nullptr)
{
    // flags: the word the multipole checks go to (the context's flag word, cleared here, when
    // NULL); a caller that passes its own has prepared the configuration already
    int rc = flags ? AMOEBA_OK : begin_config(c, pos, what);
    if (rc)
        return rc;
    if (!c->mp_d) {
        if ((rc = ctx_alloc(c, (void**)&c->mp_d, sizeof(double4) * 3 * c->npad)))
            return rc;
        if (c->mixed && (rc = ctx_alloc(c, (void**)&c->mp_f, sizeof(float4) * 3 * c->npad)))
            return rc;
    }
    // The multipole checks (finite, traceless) and the range check of the result are flags
    // written on the device and read once at the end; on an error the fields are unspecified.
    hipStream_t st = c->stream;
    if (!flags) {
        flags = c->flags;
        hipMemsetAsync(flags, 0, sizeof(int), st);
    }
    hipLaunchKernelGGL(k_gather_mpole, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, q, dip, quad,
                       c->mp_d, c->mixed ? c->mp_f : nullptr, flags);
    if (pme_use_planes(c) && !c->timing) {
        // the multipole tiles (VALU bound) on the second stream beside the reciprocal passes
        hipEventRecord(c->ev_fork, st);
        hipStreamWaitEvent(c->stream2, c->ev_fork, 0);
        if ((rc = pme_perm_potential(c)))
            return rc;
        launch_perm_tiles(c, c->stream2);
        hipEventRecord(c->ev_join, c->stream2);
        launch_gather(c, c->erec);
        hipStreamWaitEvent(st, c->ev_join, 0);
    } else {
        launch_perm_tiles(c);
        if ((rc = pme_perm_potential(c)))
            return rc;
        launch_gather(c, c->erec);
    }
    return AMOEBA_OK;
}

// Assembles E_perm with the given slot-order scales into v_q and writes it in caller order.
static void perm_field_out(amoeba_ctx* c, const double* scales, double* out)
{
    launch_perm_assemble(c, c->v_q, scales);
    if (c->mixed)
        hipLaunchKernelGGL(k_check_overflow, dim3(nblk(3 * (size_t)c->npad, 256)), dim3(256), 0, c->stream,
                           3 * (size_t)c->npad, c->v_q, kFixRange, c->flags);
    launch_scatter(c, c->v_q, out);
}

static int perm_flags_status(amoeba_ctx* c, int f, const char* what)
{
    if (f & kFlagBadCsr)
        return set_error(c, AMOEBA_E_INVALID, std::string(what) + ": quadrupole not traceless (|tr| > 1e-10)");
    if (f & kFlagNonFinite)
        return set_error(c, AMOEBA_E_NUMERIC, std::string(what) + ": non-finite multipole or field");
    if (f & kFlagOverflow)
        return set_error(c, AMOEBA_E_OVERFLOW,
                         std::string(what) + ": field outside the exact fixed-point range (|E| >= 8192 e/A^2)");
    return AMOEBA_OK;
}

static int perm_field_status(amoeba_ctx* c, const char* what)
{
    int f = 0, rc;
    if ((rc = read_flags(c, &f)))
        return rc;
    return perm_flags_status(c, f, what);
}

int amoeba_perm_field(amoeba_ctx* c, const double* pos, const double* q, const double* dip, const double* quad,
                      double* e_perm)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!q || !dip || !quad || !e_perm)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_perm_field: NULL argument");
    int rc = perm_field_parts(c, pos, q, dip, quad, "amoeba_perm_field");
    if (rc)
        return rc;
    perm_field_out(c, c->sc_s, e_perm);
    return perm_field_status(c, "amoeba_perm_field");
}

int amoeba_set_direct_scales(amoeba_ctx* c, const double* sc_s_d, int64_t n_scaled)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!c->atoms_set)
        return set_error(c, AMOEBA_E_STATE, "amoeba_set_direct_scales: call amoeba_set_atoms first");
    if (n_scaled != c->n_scaled)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_direct_scales: n_scaled differs from amoeba_set_atoms'");
    if (n_scaled > 0 && !sc_s_d)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_direct_scales: NULL sc_s_d with n_scaled > 0");
    hipStream_t st = c->stream;
    int rc;
    if (n_scaled > c->sc_sd_cap) {
        if ((rc = ctx_alloc(c, (void**)&c->sc_sd_in, sizeof(double) * n_scaled)) ||
            (rc = ctx_alloc(c, (void**)&c->sc_sd, sizeof(double) * n_scaled)))
            return rc;
        c->sc_sd_cap = n_scaled;
    }
    if (n_scaled > 0) {
        // the same validation as the p-scales: finite, and equal for both directions of a pair
        hipMemsetAsync(c->flags, 0, sizeof(int), st);
        hipLaunchKernelGGL(k_validate_atoms, dim3(nblk(c->n + 1, 256)), dim3(256), 0, st, c->n, c->alpha_in,
                           c->thole_in, c->sc_ptr_in, c->sc_j_in, sc_s_d, (long long)n_scaled, c->flags);
        int f = 0;
        if ((rc = read_flags(c, &f)))
            return rc;
        if (f & kFlagBadCsr)
            return set_error(c, AMOEBA_E_INVALID,
                             "amoeba_set_direct_scales: a non-finite scale, or a pair whose two directions "
                             "have different scales");
        hipMemcpyAsync(c->sc_sd_in, sc_s_d, sizeof(double) * n_scaled, hipMemcpyDeviceToDevice, st);
    }
    c->dscales_set = true;
    if (c->list_built && (rc = sort_params(c)))
        return rc;
    return hip_check(c, hipStreamSynchronize(st), "amoeba_set_direct_scales");
}

int amoeba_perm_field_dp(amoeba_ctx* c, const double* pos, const double* q, const double* dip, const double* quad,
                         double* e_d, double* e_p)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!q || !dip || !quad || !e_d || !e_p)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_perm_field_dp: NULL argument");
    int rc = perm_field_parts(c, pos, q, dip, quad, "amoeba_perm_field_dp");
    if (rc)
        return rc;
    perm_field_out(c, c->sc_s, e_p);
    perm_field_out(c, c->dscales_set ? c->sc_sd : c->sc_s, e_d);
    return perm_field_status(c, "amoeba_perm_field_dp");
}

int amoeba_dipole_matvec(amoeba_ctx* c, const double* pos, const double* mu, double* out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!mu || !out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_dipole_matvec: NULL argument");
    int rc = begin_config(c, pos, "amoeba_dipole_matvec");
    if (rc)
        return rc;
    if ((rc = check_vec_finite(c, mu, 3 * (size_t)c->n, "mu")))
        return rc;
    launch_gather_vec(c, mu, c->v_mu);
    launch_set_direction(c, c->v_mu);
    if ((rc = matvec_slot(c, false, false)))
        return rc;
    c->matvecs += 1;
    if ((rc = check_overflow(c, c->v_q)))
        return rc;
    launch_scatter(c, c->v_q, out);
    return hip_check(c, hipStreamSynchronize(c->stream), "amoeba_dipole_matvec");
}

int amoeba_dipole_field_parts(amoeba_ctx* c, const double* pos, const double* mu, double* e_real, double* e_recip)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!mu)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_dipole_field_parts: NULL mu");
    int rc = begin_config(c, pos, "amoeba_dipole_field_parts");
    if (rc)
        return rc;
    launch_gather_vec(c, mu, c->v_mu);
    launch_set_direction(c, c->v_mu);
    launch_mutual_tiles(c, false);
    launch_real_reduce(c, c->ereal);
    if (e_real)
        launch_scatter(c, c->ereal, e_real);
    if ((rc = pme_dipole_field(c, false)))
        return rc;
    launch_gather(c, c->erec);
    c->matvecs += 1;
    if (e_recip)
        launch_scatter(c, c->erec, e_recip);
    return hip_check(c, hipStreamSynchronize(c->stream), "amoeba_dipole_field_parts");
}

// Argument checks of the solve entry points.
static int solve_args(amoeba_ctx* c, const char* who, const double* mu_guess, int32_t guess_mode, double tol_debye,
                      int32_t max_iter)
{
    if (!(tol_debye > 0.0) || !std::isfinite(tol_debye))
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": tol_debye must be positive");
    if (max_iter < 0)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": max_iter must be >= 0");
    if (guess_mode < AMOEBA_GUESS_ZERO || guess_mode > AMOEBA_GUESS_BEST)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": unknown guess_mode");
    if (guess_mode == AMOEBA_GUESS_GIVEN && !mu_guess)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": AMOEBA_GUESS_GIVEN needs mu_guess");
    if ((guess_mode == AMOEBA_GUESS_LEARNED || guess_mode == AMOEBA_GUESS_BEST) && !c->guess_loaded)
        return set_error(c, AMOEBA_E_STATE,
                         std::string(who) + ": no learned guess model loaded (amoeba_guess_set_model)");
    return AMOEBA_OK;
}

static int polarize_body(amoeba_ctx* c, const double* mu_guess, int32_t guess_mode, double tol_debye,
                         int32_t max_iter, double* mu_out, double* e_pol_out, int32_t* iters_out);

int amoeba_polarize(amoeba_ctx* c, const double* pos, const double* e_perm, const double* mu_guess,
                    int32_t guess_mode, double tol_debye, int32_t max_iter, double* mu_out, double* e_pol_out,
                    int32_t* iters_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!e_perm || !mu_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarize: NULL e_perm or mu_out");
    int rc = solve_args(c, "amoeba_polarize", mu_guess, guess_mode, tol_debye, max_iter);
    if (rc)
        return rc;
    if ((rc = begin_config(c, pos, "amoeba_polarize")))
        return rc;
    // the inputs are checked for NaN/Inf by the gathers; the flag is read with the solve's
    // first host wait (AMOEBA_E_NUMERIC, outputs unspecified)
    hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
    launch_gather_vec_checked(c, e_perm, c->v_e);
    return polarize_body(c, mu_guess, guess_mode, tol_debye, max_iter, mu_out, e_pol_out, iters_out);
}

// The solve from the slot-order right side in v_e (the current configuration prepared).
static int polarize_body(amoeba_ctx* c, const double* mu_guess, int32_t guess_mode, double tol_debye,
                         int32_t max_iter, double* mu_out, double* e_pol_out, int32_t* iters_out)
{
    int rc;
    const bool given = mu_guess != nullptr && (guess_mode == AMOEBA_GUESS_GIVEN || guess_mode == AMOEBA_GUESS_BEST);
    c->last_guess_rms[0] = c->last_guess_rms[1] = 0.0;
    double ep = 0.0;
    int st;
    if (guess_mode == AMOEBA_GUESS_ZERO || guess_mode == AMOEBA_GUESS_GIVEN) {
        if (given)
            launch_gather_vec_checked(c, mu_guess, c->v_mu);
        st = pcg_solve(c, tol_debye, max_iter, given, mu_out, &ep);
        c->last_guess = given ? AMOEBA_GUESS_GIVEN : AMOEBA_GUESS_ZERO;
    } else if (guess_mode == AMOEBA_GUESS_LEARNED) {
        if ((rc = guess_compute(c)))
            return rc;
        guess_forward_slot(c, c->v_mu);
        st = pcg_solve(c, tol_debye, max_iter, true, mu_out, &ep);
        c->last_guess = AMOEBA_GUESS_LEARNED;
    } else {
        // Choosing the start: the preconditioned initial residual of the fallback (zero or given) and of
        // the learned guess; PCG starts from the smaller.  The fallback state is kept while
        // the learned one is evaluated.
        if ((rc = guess_compute(c)))
            return rc;
        pcg_begin(c, tol_debye);
        const size_t bytes = sizeof(double) * 3 * (size_t)c->npad;
        double rms_f = 0.0, rms_l = 0.0;
        if (given) {
            launch_gather_vec_checked(c, mu_guess, c->v_mu);
            if ((rc = pcg_start(c, true, &rms_f)))
                return rc;
            hipMemcpyAsync(c->g_save_mu, c->v_mu, bytes, hipMemcpyDeviceToDevice, c->stream);
            hipMemcpyAsync(c->g_save_q, c->v_q, bytes, hipMemcpyDeviceToDevice, c->stream);
        } else if ((rc = pcg_start(c, false, &rms_f))) {
            return rc;
        }
        guess_forward_slot(c, c->v_mu);
        if ((rc = pcg_start(c, true, &rms_l)))
            return rc;
        const bool learned = rms_l < rms_f;
        if (!learned) {
            if (given) {
                hipMemcpyAsync(c->v_mu, c->g_save_mu, bytes, hipMemcpyDeviceToDevice, c->stream);
                rc = pcg_start_from(c, c->g_save_q);
            } else {
                rc = pcg_start(c, false, nullptr);
            }
            if (rc)
                return rc;
        }
        st = pcg_run(c, max_iter, given ? 2 : 1, mu_out, &ep);
        c->last_guess = learned ? AMOEBA_GUESS_LEARNED : (given ? AMOEBA_GUESS_GIVEN : AMOEBA_GUESS_ZERO);
        c->last_guess_rms[0] = rms_f;
        c->last_guess_rms[1] = rms_l;
    }
    if (st < 0)
        return st;
    if (e_pol_out)
        *e_pol_out = ep;
    if (iters_out)
        *iters_out = c->last_iters;
    if (st == AMOEBA_NOT_CONVERGED)
        set_error(c, AMOEBA_NOT_CONVERGED, "PCG did not reach the tolerance within max_iter");
    return st;
}

int amoeba_polarize_configuration(amoeba_ctx* c, const double* pos, const double* q, const double* dip,
                                  const double* quad, const double* mu_guess, int32_t guess_mode, double tol_debye,
                                  int32_t max_iter, double* e_perm_out, double* mu_out, double* e_pol_out,
                                  int32_t* iters_out, int32_t* rebuilt_out)
{
    static const char* who = "amoeba_polarize_configuration";
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (rebuilt_out)
        *rebuilt_out = 0;
    if (!pos || !q || !dip || !quad || !mu_out)
        return set_error(c, AMOEBA_E_INVALID, std::string(who) + ": NULL pos, q, dip, quad or mu_out");
    int rc = solve_args(c, who, mu_guess, guess_mode, tol_debye, max_iter);
    if (rc)
        return rc;
    if (!c->atoms_set)
        return set_error(c, AMOEBA_E_STATE, std::string(who) + ": amoeba_set_atoms has not been called");
    // the list kept valid for pos (one host wait for the displacement test), as
    // amoeba_update_blocklist
    int32_t rebuilt = 0;
    if ((rc = amoeba_update_blocklist(c, pos, &rebuilt)))
        return rc;
    if (rebuilt_out)
        *rebuilt_out = rebuilt;
    // E_perm straight into the slot-order right side; its checks go to the second flag word,
    // read once at the end, the solve's to the first
    hipMemsetAsync(c->flags, 0, 2 * sizeof(int), c->stream);
    int* pflags = c->flags + 1;
    if ((rc = perm_field_parts(c, pos, q, dip, quad, who, pflags)))
        return rc;
    launch_perm_assemble(c, c->v_e, c->sc_s);
    if (c->mixed)
        hipLaunchKernelGGL(k_check_overflow, dim3(nblk(3 * (size_t)c->npad, 256)), dim3(256), 0, c->stream,
                           3 * (size_t)c->npad, c->v_e, kFixRange, pflags);
    if (e_perm_out)
        launch_scatter(c, c->v_e, e_perm_out);
    const int st = polarize_body(c, mu_guess, guess_mode, tol_debye, max_iter, mu_out, e_pol_out, iters_out);
    // an error of the permanent field explains any of the solve's
    hipMemcpyAsync(c->flags_host + 1, pflags, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if ((rc = hip_check(c, hipStreamSynchronize(c->stream), who)))
        return rc;
    const int f = c->flags_host[1];
    if (f) {
        c->err.clear();
        return perm_flags_status(c, f, who);
    }
    return st;
}

int amoeba_polarize_dp(amoeba_ctx* c, const double* pos, const double* e_d, const double* e_p, double tol_debye,
                       int32_t max_iter, double* mu_d_out, double* mu_p_out, double* e_pol_out, int32_t* iters_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!e_d || !e_p || !mu_d_out || !mu_p_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarize_dp: NULL e_d, e_p, mu_d_out or mu_p_out");
    if (!(tol_debye > 0.0) || !std::isfinite(tol_debye))
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarize_dp: tol_debye must be positive");
    if (max_iter < 0)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarize_dp: max_iter must be >= 0");
    int rc = begin_config(c, pos, "amoeba_polarize_dp");
    if (rc)
        return rc;
    // the d set, then the p set, each from zero with the same operator; the inputs are checked
    // for NaN/Inf by the gathers (read with each solve's first host wait)
    int st[2], it[2];
    const double* rhs[2] = {e_d, e_p};
    double* out[2] = {mu_d_out, mu_p_out};
    for (int k = 0; k < 2; ++k) {
        hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
        launch_gather_vec_checked(c, rhs[k], c->v_e);
        st[k] = pcg_solve(c, tol_debye, max_iter, false, out[k], nullptr);
        if (st[k] < 0)
            return st[k];
        it[k] = c->last_iters;
    }
    // E_pol = -1/2 C mu_d . e_p (v_e holds e_p now)
    launch_gather_vec(c, mu_d_out, c->v_mu);
    double acc = 0.0;
    if ((rc = pcg_dot_mu_e(c, &acc)))
        return rc;
    if (e_pol_out)
        *e_pol_out = -0.5 * kCoulomb * acc;
    if (iters_out) {
        iters_out[0] = it[0];
        iters_out[1] = it[1];
    }
    c->last_guess = AMOEBA_GUESS_ZERO;
    return st[0] == AMOEBA_OK && st[1] == AMOEBA_OK ? AMOEBA_OK : AMOEBA_NOT_CONVERGED;
}

int amoeba_polarization_gradient(amoeba_ctx* c, const double* pos, const double* q, const double* dip,
                                 const double* quad, const double* mu, double* grad_out)
{
    if (!c)
        return AMOEBA_E_INVALID;
    c->err.clear();
    if (!q || !dip || !quad || !mu || !grad_out)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarization_gradient: NULL argument");
    int rc = begin_config(c, pos, "amoeba_polarization_gradient");
    if (rc)
        return rc;
    if (!c->mp_d) {
        if ((rc = ctx_alloc(c, (void**)&c->mp_d, sizeof(double4) * 3 * c->npad)))
            return rc;
        if (c->mixed && (rc = ctx_alloc(c, (void**)&c->mp_f, sizeof(float4) * 3 * c->npad)))
            return rc;
    }
    hipStream_t st = c->stream;
    hipMemsetAsync(c->flags, 0, sizeof(int), st);
    hipLaunchKernelGGL(k_gather_mpole, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, q, dip, quad,
                       c->mp_d, c->mixed ? c->mp_f : nullptr, c->flags);
    launch_gather_vec_checked(c, mu, c->v_mu);
    if ((rc = polar_gradient_slot(c)))
        return rc;
    if (c->mixed)
        launch_check_overflow(c, c->ereal);   // the fixed-point pair sums
    launch_scatter(c, c->v_q, grad_out);
    int f = 0;
    if ((rc = read_flags(c, &f)))
        return rc;
    if (f & kFlagBadCsr)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_polarization_gradient: quadrupole not traceless (|tr| > 1e-10)");
    if (f & kFlagNonFinite)
        return set_error(c, AMOEBA_E_NUMERIC, "amoeba_polarization_gradient: non-finite multipole, dipole or sum");
    if (f & kFlagOverflow)
        return set_error(c, AMOEBA_E_OVERFLOW,
                         "amoeba_polarization_gradient: pair sum outside the exact fixed-point range (8192)");
    return AMOEBA_OK;
}

int amoeba_set_timing(amoeba_ctx* c, int enable)
{
    if (!c)
        return AMOEBA_E_INVALID;
    if (enable != AMOEBA_TIMING_OFF && enable != AMOEBA_TIMING_STAGES && enable != AMOEBA_TIMING_LIVE)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_timing: unknown mode");
    hipStreamSynchronize(c->stream);
    c->timing = enable == AMOEBA_TIMING_STAGES;
    c->timing_live = enable == AMOEBA_TIMING_LIVE;
    c->trec.clear();
    c->matvecs = 0;
    return AMOEBA_OK;
}

int amoeba_get_timing(amoeba_ctx* c, amoeba_timing* out)
{
    if (!c || !out)
        return AMOEBA_E_INVALID;
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "amoeba_get_timing");
    if (rc)
        return rc;
    std::memset(out, 0, sizeof(*out));
    for (auto& r : c->trec) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->tev[r.second], c->tev[r.second + 1]) != hipSuccess)
            return set_error(c, AMOEBA_E_DEVICE, "hipEventElapsedTime failed");
        out->ms[r.first] += ms;
        out->launches[r.first] += 1;
    }
    out->matvecs = c->matvecs;
    return AMOEBA_OK;
}

int amoeba_set_pme_path(amoeba_ctx* c, int32_t path)
{
    if (!c)
        return AMOEBA_E_INVALID;
    if (path != AMOEBA_PME_AUTO && path != AMOEBA_PME_PLANES && path != AMOEBA_PME_BRICKS)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_pme_path: unknown path");
    if (path == AMOEBA_PME_PLANES && !c->plane_ok)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_pme_path: the PME grid does not fit the plane path "
                                              "(K not a product of 2, 3, 5, 7, or the plane exceeds 150 KB)");
    c->pme_path = path;
    return AMOEBA_OK;
}

int amoeba_set_graphs(amoeba_ctx* c, int32_t enable)
{
    if (!c)
        return AMOEBA_E_INVALID;
    hipStreamSynchronize(c->stream);
    c->use_graphs = enable != 0;
    if (!c->use_graphs)
        iteration_graph_release(c);
    return AMOEBA_OK;
}

int amoeba_set_residual_check(amoeba_ctx* c, int32_t mode)
{
    if (!c)
        return AMOEBA_E_INVALID;
    if (mode != AMOEBA_RESIDUAL_CHECK_AUTO && mode != AMOEBA_RESIDUAL_CHECK_ALWAYS)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_residual_check: unknown mode");
    c->residual_check = mode;
    return AMOEBA_OK;
}

int amoeba_set_pair_store(amoeba_ctx* c, int32_t mode)
{
    if (!c)
        return AMOEBA_E_INVALID;
    if (mode != AMOEBA_PAIRS_AUTO && mode != AMOEBA_PAIRS_COMPUTE && mode != AMOEBA_PAIRS_STORED)
        return set_error(c, AMOEBA_E_INVALID, "amoeba_set_pair_store: unknown mode");
    c->pair_store = mode;
    if (coef_store_on(c) && c->cfg_valid && !c->coef_rows_ok)
        coef_scan_rows(c);  // the store's rows for the current masks (scanned at a refresh otherwise)
    return AMOEBA_OK;
}

int amoeba_get_info(const amoeba_ctx* cc, amoeba_info* out)
{
    if (!cc || !out)
        return AMOEBA_E_INVALID;
    amoeba_ctx* c = const_cast<amoeba_ctx*>(cc);
    if (c->pairs_pending) {
        // the pair count of the last refresh, written to pinned memory by the refresh's last
        // kernel (complete already when a call has waited for the stream since)
        if (hipEventSynchronize(c->ev_pairs) != hipSuccess)
            return AMOEBA_E_DEVICE;
        c->n_pairs = (int64_t)*c->pairs_host;
        c->pairs_pending = false;
    }
    out->n_atoms = c->n;
    out->n_blocks = c->nb;
    out->n_tiles = c->ntiles;
    out->precision = c->prm.precision;
    out->n_pairs = c->n_pairs;
    out->workspace_bytes = c->ws_bytes;
    out->last_iterations = c->last_iters;
    out->last_rms_debye = c->last_rms;
    out->last_guess = c->last_guess;
    out->guess_loaded = c->guess_loaded ? 1 : 0;
    out->last_guess_rms_debye[0] = c->last_guess_rms[0];
    out->last_guess_rms_debye[1] = c->last_guess_rms[1];
    out->pair_min_image = c->skip_mimg ? 0 : 1;
    out->pme_planes = c->plane_ok && c->pme_path != AMOEBA_PME_BRICKS ? 1 : 0;
    out->pair_store = c->coef_last_stored ? 1 : 0;
    out->pair_store_bytes = c->coef_bytes;
    return AMOEBA_OK;
}

}  // extern "C"
