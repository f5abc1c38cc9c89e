// Preconditioned conjugate gradient for the induced dipoles (paper, "Optimizations
// opportunities": PCG of the polarization solver with one matrix-vector product per iteration;
// "Performance and Scalability Results": diagonal preconditioner and convergence threshold).
//
// All vectors are FP64 in slot order (npad x 3), as are every dot product and the convergence
// test, whatever the precision of the matrix-vector product.  Scalars live on the device
// (PcgScalars): gamma and beta are computed by the last workgroup of the reductions, so an
// iteration needs no host round trip.  Once converged, a device flag makes the remaining
// queued kernels return at entry; the host reads the scalars of iteration k through an event
// while iteration k+1 is already queued.
#include "common.h"
#include "reduce.h"

namespace amoeba {

template <typename R4T> struct Cast4;
template <> struct Cast4<float4> {
    __device__ static float4 make(double x, double y, double z) { return make_float4((float)x, (float)y, (float)z, 0.f); }
};
template <> struct Cast4<double4> {
    __device__ static double4 make(double x, double y, double z) { return make_double4(x, y, z, 0.0); }
};

__global__ void k_gather_vec(int npad, const int* __restrict__ perm, const double* __restrict__ src,
                             double* __restrict__ dst)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    for (int c = 0; c < 3; ++c)
        dst[3 * (size_t)s + c] = a >= 0 ? src[3 * (size_t)a + c] : 0.0;
}

__global__ void k_scatter_vec(int npad, const int* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    if (a < 0)
        return;
    for (int c = 0; c < 3; ++c)
        dst[3 * (size_t)a + c] = src[3 * (size_t)s + c];
}

// p = src; pair-kernel copy pv = p
template <typename R4T>
__global__ void k_set_dir(int npad, const double* __restrict__ src, double* __restrict__ p, R4T* __restrict__ pv)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    double x = src[3 * (size_t)s], y = src[3 * (size_t)s + 1], z = src[3 * (size_t)s + 2];
    if (p != src) {
        p[3 * (size_t)s] = x;
        p[3 * (size_t)s + 1] = y;
        p[3 * (size_t)s + 2] = z;
    }
    pv[s] = Cast4<R4T>::make(x, y, z);
}

// r = e - q (q may be NULL: zero guess), z = alpha r, p = z; rz = r.z, rms(z) -> done?
template <typename R4T>
__global__ __launch_bounds__(256) void k_init_residual(int npad, int n, const double4* __restrict__ par,
                                                       const double* __restrict__ e, const double* __restrict__ q,
                                                       double* __restrict__ r, double* __restrict__ z,
                                                       double* __restrict__ p, R4T* __restrict__ pv,
                                                       PcgScalars* __restrict__ sc, double* part,
                                                       unsigned int* ticket)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, zz = 0.0;
    if (s < npad) {
        double al = par[s].x;
        double zv[3];
        for (int c = 0; c < 3; ++c) {
            size_t i = 3 * (size_t)s + c;
            double rv = e[i] - (q ? q[i] : 0.0);
            zv[c] = al * rv;
            r[i] = rv;
            z[i] = zv[c];
            p[i] = zv[c];
            rz += rv * zv[c];
            zz += zv[c] * zv[c];
        }
        pv[s] = Cast4<R4T>::make(zv[0], zv[1], zv[2]);
    }
    double v[2] = {rz, zz};
    grid_reduce<2>(v, part, ticket, [sc, n](const double* tot) {
        sc->rz = tot[0];
        sc->zz = tot[1];
        sc->rms = kDebye * sqrt(tot[1] / n);
        bool conv = sc->rms < sc->tol;
        sc->done = conv ? 1 : 0;
        sc->status = conv ? 1 : 0;
        if (!isfinite(tot[0])) {
            sc->done = 1;
            sc->status = 2;
        }
    });
}

// mu += gamma p, r -= gamma q, z = alpha r; rz_new = r.z, rms(z); convergence; beta
__global__ __launch_bounds__(256) void k_update(int npad, int n, const double4* __restrict__ par,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                double* __restrict__ mu, double* __restrict__ r,
                                                double* __restrict__ z, PcgScalars* __restrict__ sc, double* part,
                                                unsigned int* ticket)
{
    if (sc->done)
        return;
    const double g = sc->gamma;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double rz = 0.0, zz = 0.0;
    if (s < npad) {
        double al = par[s].x;
        for (int c = 0; c < 3; ++c) {
            size_t i = 3 * (size_t)s + c;
            mu[i] += g * p[i];
            double rv = r[i] - g * q[i];
            double zv = al * rv;
            r[i] = rv;
            z[i] = zv;
            rz += rv * zv;
            zz += zv * zv;
        }
    }
    double v[2] = {rz, zz};
    grid_reduce<2>(v, part, ticket, [sc, n](const double* tot) {
        sc->rz_new = tot[0];
        sc->zz = tot[1];
        sc->rms = kDebye * sqrt(tot[1] / n);
        sc->iters += 1;
        sc->beta = tot[0] / sc->rz;
        sc->rz = tot[0];
        if (sc->rms < sc->tol) {
            sc->done = 1;
            sc->status = 1;
        } else if (!isfinite(tot[0])) {
            sc->done = 1;
            sc->status = 2;
        }
    });
}

// p = z + beta p
template <typename R4T>
__global__ void k_direction(int npad, const double* __restrict__ z, double* __restrict__ p, R4T* __restrict__ pv,
                            const PcgScalars* __restrict__ sc)
{
    if (sc->done)
        return;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    const double b = sc->beta;
    double v[3];
    for (int c = 0; c < 3; ++c) {
        size_t i = 3 * (size_t)s + c;
        v[c] = z[i] + b * p[i];
        p[i] = v[c];
    }
    pv[s] = Cast4<R4T>::make(v[0], v[1], v[2]);
}

__global__ __launch_bounds__(256) void k_epol(int npad, const double* __restrict__ mu, const double* __restrict__ e,
                                              PcgScalars* __restrict__ sc, double* part, unsigned int* ticket)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (s < npad)
        for (int c = 0; c < 3; ++c)
            acc += mu[3 * (size_t)s + c] * e[3 * (size_t)s + c];
    double v[1] = {acc};
    grid_reduce<1>(v, part, ticket, [sc](const double* tot) { sc->epol_acc = tot[0]; });
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

void launch_gather_vec(amoeba_ctx* c, const double* src_caller, double* dst_slot)
{
    hipLaunchKernelGGL(k_gather_vec, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm, src_caller,
                       dst_slot);
}

void launch_scatter(amoeba_ctx* c, const double* v_slot, double* out_caller)
{
    hipLaunchKernelGGL(k_scatter_vec, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm, v_slot,
                       out_caller);
}

void launch_set_direction(amoeba_ctx* c, const double* src)
{
    if (c->mixed)
        hipLaunchKernelGGL(k_set_dir<float4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, src,
                           c->v_p, c->pv_f);
    else
        hipLaunchKernelGGL(k_set_dir<double4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, src,
                           c->v_p, c->pv_d);
}

// q = A p for the current direction p (pv already set); acc must be clear on entry and is clear
// on exit.
int matvec_slot(amoeba_ctx* c, bool use_done, bool dot)
{
    launch_mutual_tiles(c, use_done);
    int rc = pme_dipole_field(c, use_done);
    if (rc)
        return rc;
    launch_matvec_combine(c, use_done, dot);
    return AMOEBA_OK;
}

static void launch_init_residual(amoeba_ctx* c, const double* q)
{
    StageTimer tm(c, AMOEBA_T_PCG);
    if (c->mixed)
        hipLaunchKernelGGL(k_init_residual<float4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->n,
                           c->par_d, c->v_e, q, c->v_r, c->v_z, c->v_p, c->pv_f, c->sc, c->red.part, c->red.ticket);
    else
        hipLaunchKernelGGL(k_init_residual<double4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad,
                           c->n, c->par_d, c->v_e, q, c->v_r, c->v_z, c->v_p, c->pv_d, c->sc, c->red.part,
                           c->red.ticket);
}

static int enqueue_iteration(amoeba_ctx* c)
{
    int rc = matvec_slot(c, true, true);
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_update, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->n, c->par_d, c->v_p,
                       c->v_q, c->v_mu, c->v_r, c->v_z, c->sc, c->red.part, c->red.ticket);
    if (c->mixed)
        hipLaunchKernelGGL(k_direction<float4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->v_z,
                           c->v_p, c->pv_f, c->sc);
    else
        hipLaunchKernelGGL(k_direction<double4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->v_z,
                           c->v_p, c->pv_d, c->sc);
    return AMOEBA_OK;
}

// Iterate until the device flag says done or `budget` more iterations ran.  Host reads lag the
// device by one queued iteration.  Returns a HIP/rocFFT error code or AMOEBA_OK.
static int run_iterations(amoeba_ctx* c, int budget)
{
    hipStream_t st = c->stream;
    int enq = 0, chk = 0, rc;
    while (true) {
        if (enq < budget) {
            if ((rc = enqueue_iteration(c)))
                return rc;
            ++enq;
            hipMemcpyAsync(&c->sc_host[enq & 1], c->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, st);
            hipEventRecord(c->ev[enq & 1], st);
        }
        if (enq >= chk + 2 || enq == budget) {
            ++chk;
            if ((rc = hip_check(c, hipEventSynchronize(c->ev[chk & 1]), "pcg iteration")))
                return rc;
            if (c->sc_host[chk & 1].done || chk >= budget)
                break;
        }
    }
    return hip_check(c, hipStreamSynchronize(st), "pcg loop");
}

static int read_scalars(amoeba_ctx* c, PcgScalars* out)
{
    hipMemcpyAsync(&c->sc_host[0], c->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, c->stream);
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "read scalars");
    *out = c->sc_host[0];
    return rc;
}

// Solve A mu = e (v_e, slot order).  On entry v_mu holds the guess if have_guess.
int pcg_solve(amoeba_ctx* c, double tol, int max_iter, bool have_guess)
{
    hipStream_t st = c->stream;
    PcgScalars init{};
    init.tol = tol;
    c->sc_host[0] = init;
    hipMemcpyAsync(c->sc, &c->sc_host[0], sizeof(PcgScalars), hipMemcpyHostToDevice, st);
    int rc;
    if ((rc = hip_check(c, hipStreamSynchronize(st), "pcg init")))
        return rc;
    if (have_guess) {
        launch_set_direction(c, c->v_mu);
        if ((rc = matvec_slot(c, false, false)))
            return rc;
        launch_init_residual(c, c->v_q);
    } else {
        hipMemsetAsync(c->v_mu, 0, sizeof(double) * 3 * (size_t)c->npad, st);
        launch_init_residual(c, nullptr);
    }
    PcgScalars s;
    if ((rc = read_scalars(c, &s)))
        return rc;
    int used = 0;
    int extra_matvecs = 0;
    bool checked_true = !c->mixed;
    while (true) {
        if (!s.done && used < max_iter) {
            if ((rc = run_iterations(c, max_iter - used)))
                return rc;
            if ((rc = read_scalars(c, &s)))
                return rc;
            used = s.iters;
        }
        if (s.status == 2)
            return set_error(c, AMOEBA_E_NUMERIC, "PCG breakdown (non-positive curvature or non-finite residual)");
        if (s.status != 1 || checked_true)
            break;
        // Mixed precision: confirm convergence on the true residual e - A mu (FP64 vectors); if it
        // fails, PCG restarts from the true residual with the remaining iteration budget.
        checked_true = true;
        ++extra_matvecs;
        launch_set_direction(c, c->v_mu);
        if ((rc = matvec_slot(c, false, false)))
            return rc;
        launch_init_residual(c, c->v_q);
        PcgScalars t;
        if ((rc = read_scalars(c, &t)))
            return rc;
        t.iters = s.iters;
        s = t;
        if (s.done)
            break;
        checked_true = false;
        // restore the iteration count lost by the re-initialisation
        c->sc_host[1] = s;
        hipMemcpyAsync(c->sc, &c->sc_host[1], sizeof(PcgScalars), hipMemcpyHostToDevice, st);
        if ((rc = hip_check(c, hipStreamSynchronize(st), "pcg restart")))
            return rc;
        if (used >= max_iter)
            break;
    }
    c->last_iters = s.iters;
    c->last_rms = s.rms;
    c->matvecs += s.iters + (have_guess ? 1 : 0) + extra_matvecs;
    return s.status == 1 ? AMOEBA_OK : AMOEBA_NOT_CONVERGED;
}

double compute_epol(amoeba_ctx* c)
{
    hipLaunchKernelGGL(k_epol, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->v_mu, c->v_e, c->sc,
                       c->red.part, c->red.ticket);
    PcgScalars s;
    if (read_scalars(c, &s))
        return 0.0;
    return -0.5 * kCoulomb * s.epol_acc;
}

}  // namespace amoeba
