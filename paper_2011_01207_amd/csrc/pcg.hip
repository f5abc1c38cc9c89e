// Preconditioned conjugate gradient for the induced dipoles (paper, "Optimizations
// opportunities": PCG of the polarization solver with one matrix-vector product per iteration;
// "Performance and Scalability Results": diagonal preconditioner and convergence threshold).
//
// All vectors are FP64 in slot order (npad x 3), as are every dot product and the convergence
// test, whatever the precision of the matrix-vector product.  Scalars live on the device
// (PcgScalars): every workgroup of the kernel that needs gamma or beta sums the previous
// kernel's partials itself, so an iteration needs no host round trip.  Once converged, a
// device flag makes the remaining queued kernels return at entry; the host reads the scalars
// of iteration k through an event while iteration k+1 is already queued.  A solve waits on the
// host only for these per-iteration events and once at the end, where the outputs (E_pol, mu
// in caller order) and, in mixed precision, the true-residual check are queued together.
#include "common.h"
#include "reduce.h"

namespace amoeba {

template <typename R4T> struct Cast4;
template <> struct Cast4<float4> {
    __device__ static float4 make(double x, double y, double z, double w)
    {
        return make_float4((float)x, (float)y, (float)z, (float)w);
    }
};
template <> struct Cast4<double4> {
    __device__ static double4 make(double x, double y, double z, double w) { return make_double4(x, y, z, w); }
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

// gather that also flags a non-finite input value (checked once, at the end of the call)
__global__ void k_gather_vec_checked(int npad, const int* __restrict__ perm, const double* __restrict__ src,
                                     double* __restrict__ dst, int* __restrict__ flags)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    int a = perm[s];
    bool bad = false;
    for (int c = 0; c < 3; ++c) {
        const double v = a >= 0 ? src[3 * (size_t)a + c] : 0.0;
        bad = bad || !isfinite(v);
        dst[3 * (size_t)s + c] = v;
    }
    if (bad)
        atomicOr(flags, kFlagNonFinite);
}

__global__ void k_pcg_begin(PcgScalars* __restrict__ sc, double tol)
{
    PcgScalars init{};
    init.tol = tol;
    *sc = init;
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

// p = src; pair-kernel copy pv = p (w: the slot's Thole factor, read by the dipole tiles)
template <typename R4T>
__global__ void k_set_dir(int npad, const double4* __restrict__ par, const double* __restrict__ src,
                          double* __restrict__ p, R4T* __restrict__ pv)
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
    pv[s] = Cast4<R4T>::make(x, y, z, par[s].w);
}

// The vector kernels below use a fixed grid of kRedBlocks workgroups striding over the
// 3 npad components (component i belongs to slot i / 3); pv, the pair kernels' copy of p, is
// written component-wise.  Scalars are reduced per workgroup into partials; the next kernel
// sums the partials (see reduce.h).  Iteration `it` keeps r.z in sc->rzb[it & 1].
template <typename R4T> struct Comp;
template <> struct Comp<float4> {
    __device__ static void set(float4* v, size_t i, double x) { reinterpret_cast<float*>(v)[(i / 3) * 4 + i % 3] = (float)x; }
};
template <> struct Comp<double4> {
    __device__ static void set(double4* v, size_t i, double x) { reinterpret_cast<double*>(v)[(i / 3) * 4 + i % 3] = x; }
};

// r = e - q (q may be NULL: zero guess), z = alpha r, p = z; partials of r.z and z.z
template <typename R4T>
__global__ __launch_bounds__(256) void k_init_residual(int npad, const double* __restrict__ alpha,
                                                       const double* __restrict__ e, const double* __restrict__ q,
                                                       double* __restrict__ r, double* __restrict__ p,
                                                       R4T* __restrict__ pv, double* __restrict__ part,
                                                       int* __restrict__ range_flags)
{
    double acc[2] = {0.0, 0.0};
    bool out_of_range = false;  // the start's product, range-checked as in k_update
    const size_t n3 = 3 * (size_t)npad;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
        double al = alpha[i / 3];
        const double qi = q ? q[i] : 0.0;
        out_of_range |= !(fabs(qi) < kFixRange);
        double rv = e[i] - qi;
        double zv = al * rv;
        r[i] = rv;
        p[i] = zv;
        Comp<R4T>::set(pv, i, zv);
        acc[0] += rv * zv;
        acc[1] += zv * zv;
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
    if (range_flags && __syncthreads_or(out_of_range) && threadIdx.x == 0)
        atomicOr(range_flags, kFlagOverflow);
}

// initial scalars of iteration `it`: r.z, rms of z, converged?
__global__ __launch_bounds__(256) void k_init_finalize(int nparts, const double* __restrict__ part, int n, int it,
                                                       PcgScalars* __restrict__ sc)
{
    double tot[2];
    sum_partials<2>(part, nparts, tot);
    if (threadIdx.x == 0) {
        sc->rzb[it & 1] = tot[0];
        sc->zz = tot[1];
        sc->rms = kDebye * sqrt(tot[1] / n);
        sc->rms_sum = sc->rms;
        bool conv = sc->rms < sc->tol;
        sc->done = conv ? 1 : 0;
        sc->status = conv ? 1 : 0;
        if (!isfinite(tot[0])) {
            sc->done = 1;
            sc->status = 2;
        }
    }
}

// gamma = r.z / p.Ap (p.Ap from the gather's per-brick partials); mu += gamma p, r -= gamma Ap,
// z = alpha r; partials of the new r.z and z.z
// The iteration index is the device's count of completed iterations, so that the launches of
// an iteration take no per-iteration argument (one captured iteration serves them all).
// With integer field sums (range_flags non-NULL) every product is range-checked here: |A p| at
// or beyond kFixRange left the exact fixed-point range (AMOEBA_E_OVERFLOW at the next host read).
__global__ __launch_bounds__(256) void k_update(int npad, const double* __restrict__ alpha,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                double* __restrict__ mu, double* __restrict__ r,
                                                PcgScalars* __restrict__ sc,
                                                const double* __restrict__ part_pq, int n_pq,
                                                double* __restrict__ part, int* __restrict__ range_flags)
{
    const int it = sc->iters;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->seq_cur = sc->seq;  // for the direction kernel that follows
        sc->it_cur = it;
    }
    if (sc->done)
        return;
    double pq[1];
    sum_partials<1>(part_pq, n_pq, pq);
    if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq[0];
            sc->done = 1;
            sc->status = 2;
        }
        return;
    }
    const double g = sc->rzb[it & 1] / pq[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq[0];
        sc->gamma = g;
    }
    double acc[2] = {0.0, 0.0};
    bool out_of_range = false;
    const size_t n3 = 3 * (size_t)npad;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
        double al = alpha[i / 3];
        mu[i] += g * p[i];
        const double qi = q[i];
        out_of_range |= !(fabs(qi) < kFixRange);
        double rv = r[i] - g * qi;
        double zv = al * rv;   // z = alpha r, formed again by the direction kernel
        r[i] = rv;
        acc[0] += rv * zv;
        acc[1] += zv * zv;
    }
    block_sum<2>(acc);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
    // one device atomic per workgroup at most (same-address atomics serialize)
    if (range_flags && __syncthreads_or(out_of_range) && threadIdx.x == 0)
        atomicOr(range_flags, kFlagOverflow);
}

// convergence test on rms(z); unless converged: beta = r.z(new) / r.z(old), p = z + beta p
template <typename R4T>
__global__ __launch_bounds__(256) void k_direction(int npad, int n, const double* __restrict__ alpha,
                                                   const double* __restrict__ r, double* __restrict__ p,
                                                   R4T* __restrict__ pv,
                                                   PcgScalars* __restrict__ sc, const double* __restrict__ part,
                                                   PcgScalars* __restrict__ pub)
{
    // pub[2]: pinned host copies of the scalars, written by one thread (no separate
    // device-to-host copy per iteration); the k-th direction kernel of a solve writes pub[k & 1]
    const int it = sc->it_cur, seq = sc->seq_cur;
    if (sc->done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->seq = seq + 1;
            if (pub)
                pub[seq & 1] = *sc;
        }
        return;
    }
    double tot[2];
    sum_partials<2>(part, gridDim.x, tot);
    const double rms = kDebye * sqrt(tot[1] / n);
    const bool conv = rms < sc->tol;
    const bool bad = !isfinite(tot[0]);
    const double beta = tot[0] / sc->rzb[it & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rms = rms;
        sc->rms_sum += rms;
        sc->zz = tot[1];
        sc->iters = it + 1;
        if (conv) {
            sc->done = 1;
            sc->status = 1;
        } else if (bad) {
            sc->done = 1;
            sc->status = 2;
        } else {
            sc->rzb[(it + 1) & 1] = tot[0];
            sc->beta = beta;
        }
        sc->seq = seq + 1;
        if (pub)
            pub[seq & 1] = *sc;
    }
    if (conv || bad)
        return;
    const size_t n3 = 3 * (size_t)npad;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256) {
        double v = alpha[i / 3] * r[i] + beta * p[i];
        p[i] = v;
        Comp<R4T>::set(pv, i, v);
    }
}

__global__ __launch_bounds__(256) void k_epol(int npad, const double* __restrict__ mu, const double* __restrict__ e,
                                              double* __restrict__ part)
{
    double acc[1] = {0.0};
    const size_t n3 = 3 * (size_t)npad;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (size_t)gridDim.x * 256)
        acc[0] += mu[i] * e[i];
    block_sum<1>(acc);
    if (threadIdx.x == 0)
        part[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(256) void k_epol_finalize(int nparts, const double* __restrict__ part,
                                                       PcgScalars* __restrict__ sc)
{
    double tot[1];
    sum_partials<1>(part, nparts, tot);
    if (threadIdx.x == 0)
        sc->epol_acc = tot[0];
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

void launch_gather_vec(amoeba_ctx* c, const double* src_caller, double* dst_slot)
{
    hipLaunchKernelGGL(k_gather_vec, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm, src_caller,
                       dst_slot);
}

void launch_gather_vec_checked(amoeba_ctx* c, const double* src_caller, double* dst_slot)
{
    hipLaunchKernelGGL(k_gather_vec_checked, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm,
                       src_caller, dst_slot, c->flags);
}

void launch_scatter(amoeba_ctx* c, const double* v_slot, double* out_caller)
{
    hipLaunchKernelGGL(k_scatter_vec, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad, c->perm, v_slot,
                       out_caller);
}

void launch_set_direction(amoeba_ctx* c, const double* src)
{
    if (c->mixed)
        hipLaunchKernelGGL(k_set_dir<float4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad,
                           c->par_d, src, c->v_p, c->pv_f);
    else
        hipLaunchKernelGGL(k_set_dir<double4>, dim3(nblk(c->npad, 256)), dim3(256), 0, c->stream, c->npad,
                           c->par_d, src, c->v_p, c->pv_d);
}

// Partial buffers: the p.Ap partials of the operator product first (one per PME brick or per
// 256 atoms), then the vector kernels' [G][2].
static double* part_pq(amoeba_ctx* c) { return c->red.part; }
static double* part_vec(amoeba_ctx* c) { return c->red.part + ((size_t)c->npq_cap + 1) / 2 * 2; }

// q = A p for the current direction p (pv already set).  With the plane path the spread pass
// runs first on the whole GPU; then the real-space tiles (VALU bound) run on the second stream
// while the reciprocal transforms and the interpolation (latency bound) run on the context
// stream, so that the two share the CUs; the combine waits for both.  Stage timing keeps
// everything on the context stream so that each stage is timed alone.
// fork_ev: an event already recorded at the current end of the context stream (the PCG loop's
// per-iteration event), used as the fork point instead of recording another one.
int matvec_slot(amoeba_ctx* c, bool use_done, bool dot, hipEvent_t fork_ev)
{
    if (pme_use_planes(c) && !c->timing) {
        c->rec_plane = true;
        if (!fork_ev) {
            hipEventRecord(c->ev_fork, c->stream);
            fork_ev = c->ev_fork;
        }
        plane_dipole_field(c, use_done, 1);
        hipStreamWaitEvent(c->stream2, fork_ev, 0);
        launch_mutual_tiles(c, use_done, c->stream2);
        launch_real_reduce(c, c->ereal, c->stream2, use_done);   // E_real beside the reciprocal tail
        hipEventRecord(c->ev_join, c->stream2);
        plane_dipole_field(c, use_done, 2);
        hipStreamWaitEvent(c->stream, c->ev_join, 0);
        launch_matvec_combine(c, use_done, dot, true);
        return AMOEBA_OK;
    }
    launch_mutual_tiles(c, use_done, c->stream);
    int rc = pme_dipole_field(c, use_done);
    if (rc)
        return rc;
    launch_matvec_combine(c, use_done, dot, false);
    return AMOEBA_OK;
}

// r = e - q, z = alpha r, p = z and the scalars of iteration `it`
static void launch_init_residual(amoeba_ctx* c, const double* q, int it)
{
    StageTimer tm(c, AMOEBA_T_PCG);
    if (c->mixed)
        hipLaunchKernelGGL(k_init_residual<float4>, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->alpha_s,
                           c->v_e, q, c->v_r, c->v_p, c->pv_f, part_vec(c), c->flags);
    else
        hipLaunchKernelGGL(k_init_residual<double4>, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->alpha_s,
                           c->v_e, q, c->v_r, c->v_p, c->pv_d, part_vec(c), (int*)nullptr);
    hipLaunchKernelGGL(k_init_finalize, dim3(1), dim3(256), 0, c->stream, kRedBlocks, part_vec(c), c->n, it, c->sc);
}

static int enqueue_iteration_direct(amoeba_ctx* c, hipEvent_t fork_ev)
{
    int rc = matvec_slot(c, true, true, fork_ev);
    if (rc)
        return rc;
    StageTimer tm(c, AMOEBA_T_PCG);
    hipLaunchKernelGGL(k_update, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->alpha_s, c->v_p, c->v_q,
                       c->v_mu, c->v_r, c->sc, part_pq(c), c->npq, part_vec(c), c->mixed ? c->flags : nullptr);
    if (c->mixed)
        hipLaunchKernelGGL(k_direction<float4>, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->n,
                           c->alpha_s, c->v_r, c->v_p, c->pv_f, c->sc, part_vec(c), c->sc_host_dev);
    else
        hipLaunchKernelGGL(k_direction<double4>, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->n,
                           c->alpha_s, c->v_r, c->v_p, c->pv_d, c->sc, part_vec(c), c->sc_host_dev);
    return AMOEBA_OK;
}

void iteration_graph_release(amoeba_ctx* c)
{
    if (c->it_exec)
        hipGraphExecDestroy(c->it_exec);
    if (c->it_graph)
        hipGraphDestroy(c->it_graph);
    c->it_exec = nullptr;
    c->it_graph = nullptr;
    c->it_key = 0;
}

// What a captured iteration bakes in besides the context's fixed buffers: the pair kernel's
// minimum-image variant and coefficient mode, the coefficient store, the p.q partial count, and
// every buffer address.  A list build that outgrows its tile arrays allocates new ones (tiles,
// masks, j positions, jbuf, reverse index); the allocation registry only grows, so its size
// changes with every such allocation and a graph holding the old addresses is captured again.
static unsigned long long iteration_key(const amoeba_ctx* c)
{
    unsigned long long k = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) { k = (k ^ v) * 1099511628211ull; };
    mix((unsigned long long)c->allocs.size());
    mix((unsigned long long)c->ntiles);
    mix(c->skip_mimg ? 1 : 2);
    mix((unsigned long long)next_coef_mode(c) + 3);
    mix((unsigned long long)(uintptr_t)c->coef);
    mix((unsigned long long)c->coef_cap_rows);
    mix((unsigned long long)c->npq_cap);
    return k | 1ull;
}

// Capture one iteration on gstream (the context stream may be the legacy default stream, which
// cannot be captured); the product forks to stream2 and joins back inside the capture.
static int capture_iteration(amoeba_ctx* c)
{
    iteration_graph_release(c);
    hipStream_t saved = c->stream;
    if (hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return AMOEBA_E_DEVICE;
    }
    c->stream = c->gstream;
    int rc = enqueue_iteration_direct(c, nullptr);
    c->stream = saved;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->gstream, &g);
    if (rc || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g)
            hipGraphDestroy(g);
        return rc ? rc : AMOEBA_E_DEVICE;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        hipGraphDestroy(g);
        return AMOEBA_E_DEVICE;
    }
    c->it_graph = g;
    c->it_exec = x;
    c->it_key = iteration_key(c);
    return AMOEBA_OK;
}

// One PCG iteration: the captured graph when the overlapped plane path runs without stage timers
// and the pair coefficients are not being recorded (that launch changes host state), else the
// direct launches.  A capture that fails leaves the direct launches in use.
static int enqueue_iteration(amoeba_ctx* c, hipEvent_t fork_ev)
{
    const bool graph = c->use_graphs && !c->timing && !c->timing_live && pme_use_planes(c) && next_coef_mode(c) != 1;
    if (graph) {
        if ((!c->it_exec || c->it_key != iteration_key(c)) && capture_iteration(c) != AMOEBA_OK)
            c->use_graphs = false;
        if (c->it_exec) {
            c->rec_plane = true;  // c->npq keeps the plane path's count set during the capture
            if (hipGraphLaunch(c->it_exec, c->stream) == hipSuccess)
                return AMOEBA_OK;
            (void)hipGetLastError();
            iteration_graph_release(c);
            c->use_graphs = false;
        }
    }
    return enqueue_iteration_direct(c, fork_ev);
}

// Up to `budget` more iterations until the device flag says done (the device counts the
// iterations).  Host reads lag the device by one queued iteration; *last receives the scalars
// after the last iteration the host saw (later queued iterations return at entry).  Returns a
// HIP/rocFFT error code or AMOEBA_OK.
static int run_iterations(amoeba_ctx* c, int budget, PcgScalars* last)
{
    hipStream_t st = c->stream;
    const int seq0 = c->pcg_seq;  // the k-th iteration of this call publishes to slot (seq0 + k) & 1
    int enq = 0, chk = 0, rc;
    while (true) {
        if (enq < budget) {
            // the previous iteration's event marks the end of the stream at this point
            if ((rc = enqueue_iteration(c, enq > 0 ? c->ev[enq & 1] : nullptr)))
                return rc;
            ++enq;
            ++c->pcg_seq;
            hipEventRecord(c->ev[enq & 1], st);
        }
        if (enq >= chk + 2 || enq == budget) {
            ++chk;
            if ((rc = hip_check(c, hipEventSynchronize(c->ev[chk & 1]), "pcg iteration")))
                return rc;
            const PcgScalars& s = c->sc_host[(seq0 + chk - 1) & 1];
            if (s.done || chk >= budget) {
                *last = s;
                return AMOEBA_OK;
            }
        }
    }
}

// scalars and error flags in one round trip
static int read_state(amoeba_ctx* c, PcgScalars* out, int* flags)
{
    hipMemcpyAsync(&c->sc_host[0], c->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(c->flags_host, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "read scalars");
    *out = c->sc_host[0];
    *flags = c->flags_host[0];
    return rc;
}

static int read_scalars(amoeba_ctx* c, PcgScalars* out)
{
    int f = 0;
    int rc = read_state(c, out, &f);
    if (!rc && (f & kFlagNonFinite))
        return set_error(c, AMOEBA_E_NUMERIC, "non-finite value in e_perm, mu_guess or the guess reference");
    return rc;
}

static void launch_epol(amoeba_ctx* c)
{
    StageTimer tm(c, AMOEBA_T_PCG);
    hipLaunchKernelGGL(k_epol, dim3(kRedBlocks), dim3(256), 0, c->stream, c->npad, c->v_mu, c->v_e, part_vec(c));
    hipLaunchKernelGGL(k_epol_finalize, dim3(1), dim3(256), 0, c->stream, kRedBlocks, part_vec(c), c->sc);
}

// Sum over slots of v_mu . v_e (FP64, fixed order), waited for.
int pcg_dot_mu_e(amoeba_ctx* c, double* acc)
{
    launch_epol(c);
    PcgScalars s;
    int rc = read_scalars(c, &s);
    if (rc)
        return rc;
    *acc = s.epol_acc;
    return AMOEBA_OK;
}

// Initial device scalars of a solve (tolerance; everything else zero); no host wait.
void pcg_begin(amoeba_ctx* c, double tol)
{
    c->pcg_seq = 0;
    hipLaunchKernelGGL(k_pcg_begin, dim3(1), dim3(1), 0, c->stream, c->sc, tol);
}

// r0 = e - A mu0, z0 = alpha r0, p0 = z0 from v_mu (have_guess) or mu0 = 0.  With rms_debye
// non-NULL the host waits for the rms of z0 (and the input checks).
int pcg_start(amoeba_ctx* c, bool have_guess, double* rms_debye)
{
    int rc;
    if (have_guess) {
        launch_set_direction(c, c->v_mu);
        if ((rc = matvec_slot(c, false, false)))
            return rc;
        launch_init_residual(c, c->v_q, 0);
    } else {
        hipMemsetAsync(c->v_mu, 0, sizeof(double) * 3 * (size_t)c->npad, c->stream);
        launch_init_residual(c, nullptr, 0);
    }
    if (!rms_debye)
        return AMOEBA_OK;
    PcgScalars s;
    if ((rc = read_scalars(c, &s)))
        return rc;
    *rms_debye = s.rms;
    return AMOEBA_OK;
}

// Same with A mu0 already known (q0; NULL for mu0 = 0, v_mu must then be zero).
int pcg_start_from(amoeba_ctx* c, const double* q0)
{
    launch_init_residual(c, q0, 0);
    return AMOEBA_OK;
}

// Whether a mixed-precision solve that passed the tolerance on its recursive residual confirms
// it on the true one.  The recursion r_{k+1} = r_k - gamma_k A p_k drifts from e - A mu by the
// products' rounding, sum_k gamma_k delta(p_k); with the products' relative error below eps (the
// FP32 pair and grid arithmetic with exact integer sums: tested to 3e-6 relative rms against the
// FP64 oracle; eps is taken above three times that) and gamma_k alpha A p_k = z_k - z_{k+1}, the
// drift in z is at most 2 eps sum_k rms(z_k).  Below a tenth of the tolerance the check cannot
// change the outcome and is skipped (AMOEBA_RESIDUAL_CHECK_AUTO); ALWAYS recomputes it.
constexpr double kMixedProductRelErr = 1e-5;
constexpr double kDriftFraction = 0.1;

static bool residual_check_needed(const amoeba_ctx* c, const PcgScalars& s)
{
    return c->residual_check == AMOEBA_RESIDUAL_CHECK_ALWAYS ||
           2.0 * kMixedProductRelErr * s.rms_sum > kDriftFraction * s.tol;
}

// Iterate from the state left by pcg_start (v_mu, r, z, p and the scalars of iteration 0)
// until rms(z) < tol or max_iter iterations, then write mu (caller order) and E_pol.
// start_matvecs: products already spent on the starting point (accounting only).
int pcg_run(amoeba_ctx* c, int max_iter, int start_matvecs, double* mu_out, double* e_pol)
{
    PcgScalars s{};
    int rc, f = 0;
    int used = 0;
    int extra_matvecs = 0;
    bool checked_true = !c->mixed;
    bool first = true;
    while (true) {
        if (first || (!s.done && used < max_iter)) {
            // the first round always runs: the host has not seen the starting scalars yet (a
            // start that is already converged makes the queued kernels return at entry)
            first = false;
            if (max_iter > used) {
                if ((rc = run_iterations(c, max_iter - used, &s)))
                    return rc;
                used = s.iters;
            } else if ((rc = read_scalars(c, &s))) {
                return rc;
            }
        }
        if (s.status == 2)
            break;   // breakdown (or a non-finite input), told apart below
        // Mixed precision: confirm convergence on the true residual e - A mu (FP64 vectors) when
        // the recursion may have drifted (residual_check_needed); if it fails, PCG restarts from
        // the true residual with the remaining iteration budget.  The outputs are queued behind
        // it and kept when the check passes.
        const bool check = s.status == 1 && !checked_true && residual_check_needed(c, s);
        if (check) {
            checked_true = true;
            ++extra_matvecs;
            launch_set_direction(c, c->v_mu);
            if ((rc = matvec_slot(c, false, false)))
                return rc;
            // A mu = mu/alpha - T mu of the accepted dipoles: its fields must lie in the exact
            // fixed-point range of the tile accumulators
            launch_check_overflow(c, c->v_q);
            launch_init_residual(c, c->v_q, used);
        }
        launch_epol(c);
        launch_scatter(c, c->v_mu, mu_out);
        if ((rc = read_state(c, &s, &f)))
            return rc;
        if (f & kFlagNonFinite)
            return set_error(c, AMOEBA_E_NUMERIC, "non-finite value in e_perm, mu_guess or the guess reference");
        if (f & kFlagOverflow)
            return set_error(c, AMOEBA_E_OVERFLOW,
                             "amoeba_polarize: field outside the exact fixed-point range (|E| >= 8192 e/A^2)");
        if (check) {
            s.iters = used;
            if (!s.done) {
                checked_true = false;
                if (used < max_iter)
                    continue;
            }
        }
        break;
    }
    if (s.status == 2) {
        int fl = 0;
        if ((rc = read_state(c, &s, &fl)))
            return rc;
        if (fl & kFlagNonFinite)
            return set_error(c, AMOEBA_E_NUMERIC, "non-finite value in e_perm, mu_guess or the guess reference");
        return set_error(c, AMOEBA_E_NUMERIC, "PCG breakdown (non-positive curvature or non-finite residual)");
    }
    c->last_iters = used;
    c->last_rms = s.rms;
    c->matvecs += used + start_matvecs + extra_matvecs;
    if (e_pol)
        *e_pol = -0.5 * kCoulomb * s.epol_acc;
    return s.status == 1 ? AMOEBA_OK : AMOEBA_NOT_CONVERGED;
}

// Solve A mu = e (v_e, slot order); on entry v_mu holds the guess if have_guess.
int pcg_solve(amoeba_ctx* c, double tol, int max_iter, bool have_guess, double* mu_out, double* e_pol)
{
    pcg_begin(c, tol);
    int rc = pcg_start(c, have_guess, nullptr);
    if (rc)
        return rc;
    return pcg_run(c, max_iter, have_guess ? 1 : 0, mu_out, e_pol);
}


}  // namespace amoeba
