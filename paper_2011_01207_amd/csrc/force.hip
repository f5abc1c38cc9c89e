// Gradient of the polarization energy with respect to the atom positions (paper, "Global
// scheme": the polarization solve and its forces make the non-bonded step; "Real space scheme":
// AMOEBA's scaled pairs, corrected in a separate pass).
//
// At the converged dipoles mu = A^-1 E_perm the energy E_pol = -1/2 C mu.E_perm is stationary in
// mu, so with A = alpha^-1 - T
//     dE_pol/dr_k = C [ -1/2 mu . (dT/dr_k) mu  -  mu . dE_perm/dr_k ].
// Three passes give it:
//   * real space: the ForceKind tiles (realspace.hip), sum_j G_ij per atom, unscaled pairs;
//   * the scaled-pair correction (k_force_scaled, FP64): each listed pair's G with the radial
//     functions of the scale minus those the tiles used (inside rc), or the bare scaled tensors
//     (beyond rc, where the tiles skipped the pair);
//   * reciprocal space (k_force_recip): with Q_mu the spread of the dipoles and Q_p that of the
//     multipoles and psi_x = theta * Q_x their grid potentials (theta symmetric),
//       dE_pol,rec/dr_m = C sum_k [ dQ_mu/dr_m (psi_mu + psi_p) + dQ_p/dr_m psi_mu ],
//     where dQ_mu/dr_m needs the second and dQ_p/dr_m the third B-spline derivatives.
// The dipole self terms do not depend on the positions.
#include "common.h"
#include "spline.h"

namespace amoeba {

// [npad][4] R4 source of the ForceKind tiles: the three multipole records and the dipoles.
template <typename R4T>
__global__ void k_force_src(int npad, const double4* __restrict__ mp, const double* __restrict__ mu,
                            R4T* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    using RT = decltype(out->x);
    for (int k = 0; k < 3; ++k) {
        const double4 m = mp[3 * (size_t)s + k];
        out[4 * (size_t)s + k] = R4T{(RT)m.x, (RT)m.y, (RT)m.z, (RT)m.w};
    }
    out[4 * (size_t)s + 3] = R4T{(RT)mu[3 * (size_t)s], (RT)mu[3 * (size_t)s + 1], (RT)mu[3 * (size_t)s + 2], (RT)0};
}

// grad_r of w = mu . E_mp(r) for the multipole (q, d, Theta) of slot j (FP64).
__device__ __forceinline__ void grad_w64(const double* m3, const double4* mp, int j, const double r[3],
                                         const double b[5], double g[3])
{
    const double4 m0 = mp[3 * (size_t)j], m1 = mp[3 * (size_t)j + 1], m2 = mp[3 * (size_t)j + 2];
    const double q = m0.x, d[3] = {m0.y, m0.z, m0.w};
    const double th[3][3] = {{m1.x, m1.y, m1.z}, {m1.y, m1.w, m2.x}, {m1.z, m2.x, m2.y}};
    const double mr = m3[0] * r[0] + m3[1] * r[1] + m3[2] * r[2];
    const double dr = d[0] * r[0] + d[1] * r[1] + d[2] * r[2];
    const double md = m3[0] * d[0] + m3[1] * d[1] + m3[2] * d[2];
    double thr[3], thm[3];
    for (int a = 0; a < 3; ++a) {
        thr[a] = th[a][0] * r[0] + th[a][1] * r[1] + th[a][2] * r[2];
        thm[a] = th[a][0] * m3[0] + th[a][1] * m3[1] + th[a][2] * m3[2];
    }
    const double thrr = thr[0] * r[0] + thr[1] * r[1] + thr[2] * r[2];
    const double mthr = m3[0] * thr[0] + m3[1] * thr[1] + m3[2] * thr[2];
    for (int a = 0; a < 3; ++a)
        g[a] = q * (b[1] * m3[a] - b[2] * mr * r[a]) + b[2] * md * r[a] + b[2] * (d[a] * mr + m3[a] * dr) -
               b[3] * dr * mr * r[a] + (b[3] * (2.0 * thr[a] * mr + thrr * m3[a]) - b[4] * thrr * mr * r[a]) / 3.0 -
               2.0 * (b[2] * thm[a] - b[3] * mthr * r[a]) / 3.0;
}

// Scaled-pair correction of the gradient, per slot over its listed partners (FP64):
//   inside rc:  delta B_n = -c_n (1 - s) lambda_{2n+1} / r^{2n+1}   (the tiles used s = 1)
//   beyond rc:  delta B_n = -c_n (1 - s lambda_{2n+1}) / r^{2n+1}   (the tiles skipped the pair)
// out[s] = sum over the listed j of grad w_sj(r) - (grad w_js)(-r) with these delta B_n.
__global__ void k_force_scaled(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                               const double4* __restrict__ par, const double4* __restrict__ mp,
                               const double* __restrict__ mu, const int* __restrict__ sc_ptr,
                               const int* __restrict__ sc_j, const double* __restrict__ sc_s, double3 box,
                               double3 binv, double rc2, double* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    double acc[3] = {0.0, 0.0, 0.0};
    if (perm[s] >= 0) {
        const double4 pi = pos_s[s], pari = par[s];
        const double mi[3] = {mu[3 * (size_t)s], mu[3 * (size_t)s + 1], mu[3 * (size_t)s + 2]};
        for (int k = sc_ptr[s]; k < sc_ptr[s + 1]; ++k) {
            const int j = sc_j[k];
            const double sf = sc_s[k];
            const double4 pj = pos_s[j], parj = par[j];
            double r[3] = {mimg_fp64(pi.x - pj.x, box.x, binv.x), mimg_fp64(pi.y - pj.y, box.y, binv.y),
                           mimg_fp64(pi.z - pj.z, box.z, binv.z)};
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const bool in = r2 < rc2;
            if (in && sf == 1.0)
                continue;
            const double rn = sqrt(r2), rinv = 1.0 / rn, rinv2 = rinv * rinv;
            const double a = fmin(pari.w, parj.w);
            const double u = rn * pari.z * parj.z;
            const double eps = a * u * u * u;
            const double ex = exp(-eps);
            const double lam[5] = {0.0, 1.0 - ex, 1.0 - (1.0 + eps) * ex, 1.0 - (1.0 + eps + 0.6 * eps * eps) * ex,
                                   1.0 - (1.0 + eps + (18.0 / 35.0) * eps * eps + (9.0 / 35.0) * eps * eps * eps) * ex};
            const double cn[5] = {0.0, 1.0, 3.0, 15.0, 105.0};
            double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            double rp = rinv * rinv2;
            for (int n = 1; n <= 4; ++n) {
                b[n] = in ? -cn[n] * (1.0 - sf) * lam[n] * rp : -cn[n] * (1.0 - sf * lam[n]) * rp;
                rp *= rinv2;
            }
            const double mj[3] = {mu[3 * (size_t)j], mu[3 * (size_t)j + 1], mu[3 * (size_t)j + 2]};
            double g[3];
            grad_w64(mi, mp, j, r, b, g);
            for (int c = 0; c < 3; ++c)
                acc[c] += g[c];
            const double mr[3] = {-r[0], -r[1], -r[2]};
            grad_w64(mj, mp, s, mr, b, g);
            for (int c = 0; c < 3; ++c)
                acc[c] -= g[c];
        }
    }
    for (int c = 0; c < 3; ++c)
        out[3 * (size_t)s + c] = acc[c];
}

// Order-5 B-spline values and derivatives up to the third at M5(w + t), t = 0..4 (Essmann et al.
// 1995: M_n(x) = (x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)) / (n - 1); the k-th derivative of M5 is
// the k-th difference of M_{5-k}).
__device__ __forceinline__ void spline5_d3(double w, double m[4][5])
{
    double a2[5] = {w, 1.0 - w, 0.0, 0.0, 0.0};   // M2(w + t)
    double a3[5], a4[5], a5[5];
    auto raise = [&](const double* lo, double* hi, int k) {
        for (int t = 0; t < 5; ++t)
            hi[t] = ((w + t) * lo[t] + ((double)k - w - t) * (t > 0 ? lo[t - 1] : 0.0)) / (k - 1);
    };
    raise(a2, a3, 3);
    raise(a3, a4, 4);
    raise(a4, a5, 5);
    for (int t = 0; t < 5; ++t) {
        const double l1 = t > 0 ? 1.0 : 0.0, l2 = t > 1 ? 1.0 : 0.0, l3 = t > 2 ? 1.0 : 0.0;
        m[0][t] = a5[t];
        m[1][t] = a4[t] - l1 * a4[t > 0 ? t - 1 : 0];
        m[2][t] = a3[t] - 2.0 * l1 * a3[t > 0 ? t - 1 : 0] + l2 * a3[t > 1 ? t - 2 : 0];
        m[3][t] = a2[t] - 3.0 * l1 * a2[t > 0 ? t - 1 : 0] + 3.0 * l2 * a2[t > 1 ? t - 2 : 0] -
                  l3 * a2[t > 2 ? t - 3 : 0];
    }
}

// Reciprocal part and assembly, one thread per slot:
//   rec = sum over the atom's 125 grid points of
//         psi_a(k) (H mu) + psi_b(k) (q grad W + H d + 1/3 sum_bc Theta_bc d_a d_b d_c W),
//   H_ab = d_a d_b W, psi_a = psi_mu + psi_p, psi_b = psi_mu;
//   grad = C (rec - real - corr)   (real, corr: the pair sums of the two other passes).
template <typename R>
__global__ void k_force_recip(int npad, const int* __restrict__ perm, const double4* __restrict__ pos_s,
                              double3 kl, int3 K, const R* __restrict__ psi_mu, const R* __restrict__ psi_p,
                              const double4* __restrict__ mp, const double* __restrict__ mu,
                              const double* __restrict__ real, const double* __restrict__ corr,
                              double* __restrict__ grad)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad)
        return;
    if (perm[s] < 0) {
        grad[3 * (size_t)s] = grad[3 * (size_t)s + 1] = grad[3 * (size_t)s + 2] = 0.0;
        return;
    }
    const double4 p = pos_s[s];
    int f[3];
    double w[3];
    grid_coord(p.x, kl.x, K.x, f[0], w[0]);
    grid_coord(p.y, kl.y, K.y, f[1], w[1]);
    grid_coord(p.z, kl.z, K.z, f[2], w[2]);
    const double klv[3] = {kl.x, kl.y, kl.z};
    const int Kv[3] = {K.x, K.y, K.z};
    double m[3][4][5];
    int g[3][5];
    for (int a = 0; a < 3; ++a) {
        spline5_d3(w[a], m[a]);
        double sc = 1.0;
        for (int d = 0; d < 4; ++d) {
            for (int t = 0; t < 5; ++t)
                m[a][d][t] *= sc;
            sc *= klv[a];
        }
        for (int t = 0; t < 5; ++t) {
            const int v = f[a] - t;
            g[a][t] = v < 0 ? v + Kv[a] : v;
        }
    }
    const double4 m0 = mp[3 * (size_t)s], m1 = mp[3 * (size_t)s + 1], m2 = mp[3 * (size_t)s + 2];
    const double q = m0.x, d[3] = {m0.y, m0.z, m0.w};
    const double th[3][3] = {{m1.x, m1.y, m1.z}, {m1.y, m1.w, m2.x}, {m1.z, m2.x, m2.y}};
    const double mi[3] = {mu[3 * (size_t)s], mu[3 * (size_t)s + 1], mu[3 * (size_t)s + 2]};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int tx = 0; tx < 5; ++tx)
        for (int ty = 0; ty < 5; ++ty) {
            const size_t row = ((size_t)g[0][tx] * K.y + g[1][ty]) * K.z;
            for (int tz = 0; tz < 5; ++tz) {
                const double pm = (double)psi_mu[row + g[2][tz]];
                const double pa = pm + (double)psi_p[row + g[2][tz]];
                const int tt[3] = {tx, ty, tz};
                // W derivative of orders (ox, oy, oz)
                auto W = [&](int ox, int oy, int oz) { return m[0][ox][tt[0]] * m[1][oy][tt[1]] * m[2][oz][tt[2]]; };
                for (int x = 0; x < 3; ++x) {
                    int o1[3] = {x == 0, x == 1, x == 2};
                    double hm = 0.0, hd = 0.0, t3 = 0.0;
                    for (int y = 0; y < 3; ++y) {
                        const int o2[3] = {o1[0] + (y == 0), o1[1] + (y == 1), o1[2] + (y == 2)};
                        const double h = W(o2[0], o2[1], o2[2]);
                        hm += h * mi[y];
                        hd += h * d[y];
                        for (int z = 0; z < 3; ++z)
                            t3 += th[y][z] * W(o2[0] + (z == 0), o2[1] + (z == 1), o2[2] + (z == 2));
                    }
                    acc[x] += pa * hm + pm * (q * W(o1[0], o1[1], o1[2]) + hd + t3 / 3.0);
                }
            }
        }
    for (int c = 0; c < 3; ++c)
        grad[3 * (size_t)s + c] = kCoulomb * (acc[c] - real[3 * (size_t)s + c] - corr[3 * (size_t)s + c]);
}

static inline int nblk(size_t n, int b) { return (int)((n + b - 1) / b); }

// dE_pol/dr in slot order into c->v_q, for the multipoles in mp_d/mp_f and the dipoles in v_mu
// (both gathered by the caller).  Uses the brick spread and rocFFT for the two grid potentials.
int polar_gradient_slot(amoeba_ctx* c)
{
    hipStream_t st = c->stream;
    int rc;
    const size_t rs = c->mixed ? sizeof(float) : sizeof(double);
    if (!c->f_src) {
        if ((rc = ctx_alloc(c, &c->f_src, 4 * 4 * rs * (size_t)c->npad)) ||
            (rc = ctx_alloc(c, &c->f_psi, rs * c->ngrid)))
            return rc;
    }
    // sources: ForceKind records (multipoles + dipoles) and the pair kernels' dipole copy
    if (c->mixed)
        hipLaunchKernelGGL(k_force_src<float4>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->mp_d,
                           c->v_mu, (float4*)c->f_src);
    else
        hipLaunchKernelGGL(k_force_src<double4>, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->mp_d,
                           c->v_mu, (double4*)c->f_src);
    launch_set_direction(c, c->v_mu);
    // real space: sum_j G_ij into ereal
    launch_force_tiles(c, c->f_src, c->ereal);
    // scaled pairs: into erec
    {
        double3 box = make_double3(c->prm.box[0], c->prm.box[1], c->prm.box[2]);
        hipLaunchKernelGGL(k_force_scaled, dim3(nblk(c->npad, 256)), dim3(256), 0, st, c->npad, c->perm, c->pos_s,
                           c->par_d, (const double4*)c->mp_d, c->v_mu, c->sc_ptr, c->sc_j, c->sc_s, box,
                           make_double3(1.0 / box.x, 1.0 / box.y, 1.0 / box.z), c->prm.cutoff * c->prm.cutoff,
                           c->erec);
    }
    // grid potentials: psi_p (multipoles) kept in f_psi, then psi_mu (dipoles) in grid_r
    if ((rc = pme_brick_potential(c, true)))
        return rc;
    hipMemcpyAsync(c->f_psi, c->grid_r, rs * c->ngrid, hipMemcpyDeviceToDevice, st);
    if ((rc = pme_brick_potential(c, false)))
        return rc;
    int3 K = make_int3(c->K[0], c->K[1], c->K[2]);
    double3 kl = make_double3(c->K[0] / c->prm.box[0], c->K[1] / c->prm.box[1], c->K[2] / c->prm.box[2]);
    if (c->mixed)
        hipLaunchKernelGGL(k_force_recip<float>, dim3(nblk(c->npad, 128)), dim3(128), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, (const float*)c->grid_r, (const float*)c->f_psi,
                           (const double4*)c->mp_d, c->v_mu, c->ereal, c->erec, c->v_q);
    else
        hipLaunchKernelGGL(k_force_recip<double>, dim3(nblk(c->npad, 128)), dim3(128), 0, st, c->npad, c->perm,
                           c->pos_s, kl, K, (const double*)c->grid_r, (const double*)c->f_psi,
                           (const double4*)c->mp_d, c->v_mu, c->ereal, c->erec, c->v_q);
    return AMOEBA_OK;
}

}  // namespace amoeba
