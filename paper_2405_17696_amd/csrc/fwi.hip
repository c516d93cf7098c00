// Data misfit of eq. (3.5) (identity covariance) and its gradient with respect
// to the squared slowness, by one forward and one adjoint solve per
// (frequency, source); the adjoint solve uses the conjugation identity of
// eq. (4.8).  The solves are batched through helm_solve: all frequencies and
// sources of the call go into one ragged launch.
//
//   u_fs      = H_f^{-1} g_s,             g_s = e_src(s) / (hx hz)
//   res_fs    = R u_fs - d_fs              (R: sample at the receiver nodes)
//   Phi       = 1/2 sum_fs |res_fs|^2
//   lambda_fs = H_f^{-*} R^T res_fs
//   dPhi/dm_k = sum_f w_f^2 sum_s Re( conj(lambda_fs[k]) (1 - i gamma_k) u_fs[k] )
//
// The last line follows from dH_f/dm_k = -w_f^2 (1 - i gamma_k) e_k e_k^T
// (eq. 3.1); the Jacobian printed with eq. (3.10) carries the opposite sign.
//
// Simultaneous sources (Sec. 3.2, eq. 3.6-3.8): with an ns x p matrix X of
// Rademacher columns (drawn by the caller), the frequency's source sum is
// replaced by the trace estimate (1/p) sum_i || R H_f^{-1} G x_i - D_f x_i ||^2:
// p encoded sources G x_i and encoded data D_f x_i take the place of the ns
// point sources and their data, and misfit and gradient carry the factor 1/p.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace helm {

namespace {

__global__ void k_point_sources(const int* __restrict__ src, int ns, int nfs, long N, float amp, c64* __restrict__ rhs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfs) return;
    rhs[(long)t * N + src[t % ns]] = c64{amp, 0.f};
}

// Encoded sources into the zeroed rhs: rhs_(f,i) = amp sum_s X[s][i] e_src(s),
// one thread per (f, i) adding the sources in order (coinciding source nodes
// add up).
__global__ void k_encoded_sources(const int* __restrict__ src, const float* __restrict__ X, int ns, int p, int nfp,
                                  long N, float amp, c64* __restrict__ rhs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfp) return;
    const int i = t % p;
    c64* r = rhs + (long)t * N;
    for (int s = 0; s < ns; ++s) {
        c64 v = r[src[s]];
        v.re += amp * X[(long)s * p + i];
        r[src[s]] = v;
    }
}

// Encoded data dx[f][i][r] = sum_s X[s][i] dobs[f][s][r], summed in FP64 in
// source order and stored as c64.
__global__ void k_encode_data(const c64* __restrict__ dobs, const float* __restrict__ X, int ns, int p, int nrec,
                              long total, c64* __restrict__ dx) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int r = (int)(t % nrec);
    const long fi = t / nrec;
    const int i = (int)(fi % p), f = (int)(fi / p);
    double re = 0, im = 0;
    for (int s = 0; s < ns; ++s) {
        const c64 d = dobs[((long)f * ns + s) * nrec + r];
        const double w = X[(long)s * p + i];
        re += w * d.re;
        im += w * d.im;
    }
    dx[t] = c64{(float)re, (float)im};
}

// One block per (f, s): residual at the receivers (FP64), the adjoint source
// R^T res written into the zeroed rhs, and 1/2 |res|^2 folded in a fixed order.
__global__ __launch_bounds__(256) void k_fwi_residual(const c128* __restrict__ u, const c64* __restrict__ dobs,
                                                      const int* __restrict__ rec, int nrec, long N,
                                                      c64* __restrict__ rhs, double* __restrict__ part) {
    __shared__ double red[256];
    const int fs = blockIdx.x, tid = threadIdx.x;
    double acc = 0;
    for (int r = tid; r < nrec; r += 256) {
        const c128 v = u[(long)fs * N + rec[r]];
        const c64 d = dobs[(long)fs * nrec + r];
        const double re = v.re - (double)d.re, im = v.im - (double)d.im;
        rhs[(long)fs * N + rec[r]] = c64{(float)re, (float)im};
        acc += re * re + im * im;
    }
    red[tid] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) part[fs] = 0.5 * red[0];
}

// gacc[k] (+)= w^2 sum_s Re(conj(lam_s[k]) (1 - i gamma_k) u_s[k]) for one frequency.
__global__ void k_fwi_grad_freq(const c128* __restrict__ u, const c128* __restrict__ lam, const float* __restrict__ gam,
                                double w2, int ns, long N, int first, double* __restrict__ gacc) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double g = gam[k];
    double acc = 0;
    for (int s = 0; s < ns; ++s) {
        const c128 a = u[(long)s * N + k], l = lam[(long)s * N + k];
        // (1 - i g) u = (u.re + g u.im) + i (u.im - g u.re)
        acc += l.re * (a.re + g * a.im) + l.im * (a.im - g * a.re);
    }
    gacc[k] = first ? w2 * acc : gacc[k] + w2 * acc;
}

// Born sources of one frequency: rhs_s = w^2 (1 - i gamma) u_s dm (c64), nper fields.
__global__ void k_born_source(const c128* __restrict__ u, const float* __restrict__ gam, const float* __restrict__ dm,
                              double w2, int nper, long N, c64* __restrict__ rhs) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double g = gam[k], d = w2 * (double)dm[k];
    for (int s = 0; s < nper; ++s) {
        const c128 a = u[(long)s * N + k];
        // (1 - i g) u = (u.re + g u.im) + i (u.im - g u.re)
        rhs[(long)s * N + k] = c64{(float)(d * (a.re + g * a.im)), (float)(d * (a.im - g * a.re))};
    }
}

// out[fs][r] = field fs at receiver r (c64).
__global__ void k_sample_rec(const c128* __restrict__ u, const int* __restrict__ rec, int nrec, long N, long total,
                             c64* __restrict__ out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const c128 v = u[(t / nrec) * N + rec[t % nrec]];
    out[t] = c64{(float)v.re, (float)v.im};
}

// R^T dd into the zeroed rhs: rhs[fs][rec[r]] = dd[fs][r].
__global__ void k_scatter_rec(const c64* __restrict__ dd, const int* __restrict__ rec, int nrec, long N, long total,
                              c64* __restrict__ rhs) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    rhs[(t / nrec) * N + rec[t % nrec]] = dd[t];
}

// Conjugate-gradient vector work in FP64.  Dot products: CG_BLOCKS fixed blocks
// sum fixed strided ranges in order and fold in a tree; the host adds the block
// partials in order, so every run gives the same bits.
constexpr int CG_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_cg_dot(const double* __restrict__ a, const double* __restrict__ b, long n,
                                                double* __restrict__ part) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double acc = 0;
    for (long k = (long)blockIdx.x * 256 + tid; k < n; k += (long)CG_BLOCKS * 256) acc += a[k] * b[k];
    red[tid] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = red[0];
}

__global__ void k_f2d_scaled(const float* __restrict__ a, double sign, long n, double* __restrict__ b) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = sign * (double)a[t];
}

// m_new = m + mu dm (FP32 model arrays; m_new may alias m)
__global__ void k_model_update(const float* m, const float* __restrict__ dm, double mu, long n, float* m_new) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) m_new[t] = (float)((double)m[t] + mu * (double)dm[t]);
}

// ap = hp + damping p
__global__ void k_cg_ap(const float* __restrict__ hp, const double* __restrict__ p, double damping, long n,
                        double* __restrict__ ap) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) ap[t] = (double)hp[t] + damping * p[t];
}

// x += alpha p, r -= alpha ap
__global__ void k_cg_xr(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                        const double* __restrict__ ap, double alpha, long n) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    x[t] += alpha * p[t];
    r[t] -= alpha * ap[t];
}

// p = r + beta p
__global__ void k_cg_p(double* __restrict__ p, const double* __restrict__ r, double beta, long n) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = r[t] + beta * p[t];
}

__global__ void k_to_float(const double* __restrict__ a, long n, float* __restrict__ b) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

struct Owned {
    std::vector<void*> p;
    ~Owned() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        p.push_back(q);
        return (T*)q;
    }
};

// Checks shared by both entry points.
static int check_args(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                      const int* rec_idx, int nrec) {
    for (int f = 0; f < nfreq; ++f) {
        if (!ops[f]) return fail(HELM_EINVAL, "%s: ops[%d] is NULL", name, f);
        const helm_op* a = ops[f];
        const helm_op* b = ops[0];
        if (a->nz != b->nz || a->nx != b->nx || a->hx != b->hx || a->hz != b->hz)
            return fail(HELM_EINVAL, "%s: operator %d is on a different grid", name, f);
    }
    const long N = ops[0]->n();
    for (int i = 0; i < nsrc; ++i)
        if (src_idx[i] < 0 || src_idx[i] >= N) return fail(HELM_EINVAL, "%s: source %d out of range", name, i);
    std::vector<int> rs(rec_idx, rec_idx + nrec);
    std::sort(rs.begin(), rs.end());
    for (int i = 0; i < nrec; ++i) {
        if (rs[i] < 0 || rs[i] >= N) return fail(HELM_EINVAL, "%s: receiver index out of range", name);
        if (i && rs[i] == rs[i - 1]) return fail(HELM_EINVAL, "%s: receiver nodes must be distinct", name);
    }
    return HELM_OK;
}

// From nper prepared right-hand sides per frequency (rhs, zero outside the
// sources) and their data dobs_d [nfreq][nper][nrec] (device): forward solves,
// residuals and misfit, adjoint solves, gradient; misfit and gradient times scale.
static int misfit_grad_core(const helm_op_t* ops, int nfreq, int nper, c64* rhs, const c64* dobs_d,
                            const int* rec_d, int nrec, double tol, helm_solve_opts o, double scale, double* misfit,
                            float* grad, int* iters, hipStream_t s, Owned& own, c128* u_keep = nullptr) {
    const long N = ops[0]->n();
    const int nfs = nfreq * nper;
    c128* u = u_keep ? u_keep : own.get<c128>((size_t)nfs * N);   // u_keep: the caller keeps the fields
    c128* lam = own.get<c128>((size_t)nfs * N);
    double* gacc = own.get<double>(N);
    double* part = own.get<double>(nfs);
    if (!u || !lam || !gacc || !part) return fail(HELM_ENOMEM, "fwi_misfit_grad: workspace allocation failed");
    std::vector<int> rhs_op(nfs);
    for (int i = 0; i < nfs; ++i) rhs_op[i] = i / nper;
    std::vector<int> st(nfs), it(nfs);

    // forward solves
    int rc = helm_solve(ops, nfreq, rhs_op.data(), rhs, u, nfs, tol, &o, it.data(), nullptr, st.data(), s);
    if (rc < 0) return rc;
    int worst = rc;
    if (iters) std::copy(it.begin(), it.end(), iters);

    // residuals, misfit, adjoint sources
    HELM_HIP(hipMemsetAsync(rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
    hipLaunchKernelGGL(k_fwi_residual, dim3(nfs), dim3(256), 0, s, u, dobs_d, rec_d, nrec, N, rhs, part);
    HELM_CHECK_LAUNCH();
    std::vector<double> ph(nfs);
    HELM_HIP(hipMemcpyAsync(ph.data(), part, sizeof(double) * nfs, hipMemcpyDeviceToHost, s));

    // adjoint solves: lambda = H^{-*} R^T res
    o.adjoint = 1;
    rc = helm_solve(ops, nfreq, rhs_op.data(), rhs, lam, nfs, tol, &o, it.data(), nullptr, st.data(), s);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    if (iters) std::copy(it.begin(), it.end(), iters + nfs);

    // gradient, frequency by frequency in a fixed order
    const int nb = (int)((N + 255) / 256);
    for (int f = 0; f < nfreq; ++f) {
        const double w2 = ops[f]->omega * ops[f]->omega * scale;
        hipLaunchKernelGGL(k_fwi_grad_freq, dim3(nb), dim3(256), 0, s, u + (size_t)f * nper * N,
                           lam + (size_t)f * nper * N, (const float*)ops[f]->lv[0].g, w2, nper, N, f == 0 ? 1 : 0,
                           gacc);
        HELM_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, gacc, N, grad);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipStreamSynchronize(s));
    double phi = 0;
    for (int i = 0; i < nfs; ++i) phi += ph[i];
    *misfit = phi * scale;
    return worst == HELM_NOT_CONVERGED ? HELM_NOT_CONVERGED : HELM_OK;
}

// Workspace of the linearised products: rhs (c64) and u, w (c128) per (f, s),
// receiver data (c64) and the FP64 gradient accumulator.
struct BornWork {
    c64* rhs = nullptr;
    c128* u = nullptr;
    c128* w = nullptr;
    c64* jd = nullptr;
    double* gacc = nullptr;
};

static int born_alloc(Owned& own, long N, int nfs, long nd, BornWork& W) {
    W.rhs = own.get<c64>((size_t)nfs * N);
    W.u = own.get<c128>((size_t)nfs * N);
    W.w = own.get<c128>((size_t)nfs * N);
    W.jd = own.get<c64>((size_t)nd);
    W.gacc = own.get<double>(N);
    if (!W.rhs || !W.u || !W.w || !W.jd || !W.gacc) return fail(HELM_ENOMEM, "fwi born: workspace allocation failed");
    return HELM_OK;
}

// Linearised data and its adjoint (eq. 3.10, with the sign derived from
// eq. 3.1): from the point-source fields u_fs (computed into W.u unless
// have_u),
//   J dm      = R H_f^{-1} (w_f^2 (1 - i gamma) u_fs dm)          (when dm != NULL)
//   Re(J^H d) = sum_fs w_f^2 Re(conj(H_f^{-*} R^T d_fs) (1 - i gamma) u_fs)
// with d = dd, or d = J dm when dd is NULL (the Gauss-Newton product).  jdm
// (device c64 [nfreq][nsrc][nrec], may be NULL) receives J dm, out (device
// float [nz][nx], may be NULL) Re(J^H d); iters receives one [nfreq][nsrc]
// block per solve batch in the order forward, Born, adjoint.
static int born_core(const helm_op_t* ops, int nfreq, int nsrc, const int* src_d, const int* rec_d, int nrec,
                     const float* dm, const c64* dd, c64* jdm, float* out, double tol, helm_solve_opts o, int* iters,
                     hipStream_t s, const BornWork& W, bool have_u) {
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    const long nd = (long)nfs * nrec;
    c64* jd = jdm ? jdm : W.jd;
    std::vector<int> rhs_op(nfs);
    for (int i = 0; i < nfs; ++i) rhs_op[i] = i / nsrc;
    std::vector<int> st(nfs), it(nfs);
    int worst = HELM_OK, stage = 0;
    auto solve = [&](c128* x, int adjoint) {
        o.adjoint = adjoint;
        const int rc =
            helm_solve(ops, nfreq, rhs_op.data(), W.rhs, x, nfs, tol, &o, it.data(), nullptr, st.data(), s);
        if (rc >= 0) {
            worst = std::max(worst, rc);
            if (iters) std::copy(it.begin(), it.end(), iters + (size_t)stage * nfs);
            ++stage;
        }
        return rc;
    };
    const unsigned gd = (unsigned)((nd + 255) / 256);
    const int nb = (int)((N + 255) / 256);
    int rc;

    // point-source fields
    if (!have_u) {
        HELM_HIP(hipMemsetAsync(W.rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
        const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
        hipLaunchKernelGGL(k_point_sources, dim3((nfs + 255) / 256), dim3(256), 0, s, src_d, nsrc, nfs, N, amp,
                           W.rhs);
        HELM_CHECK_LAUNCH();
        if ((rc = solve(W.u, 0)) < 0) return rc;
    }

    // J dm
    if (dm) {
        for (int f = 0; f < nfreq; ++f) {
            hipLaunchKernelGGL(k_born_source, dim3(nb), dim3(256), 0, s, W.u + (size_t)f * nsrc * N,
                               (const float*)ops[f]->lv[0].g, dm, ops[f]->omega * ops[f]->omega, nsrc, N,
                               W.rhs + (size_t)f * nsrc * N);
            HELM_CHECK_LAUNCH();
        }
        if ((rc = solve(W.w, 0)) < 0) return rc;
        hipLaunchKernelGGL(k_sample_rec, dim3(gd), dim3(256), 0, s, W.w, rec_d, nrec, N, nd, jd);
        HELM_CHECK_LAUNCH();
    }

    // Re(J^H d)
    if (out) {
        HELM_HIP(hipMemsetAsync(W.rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
        hipLaunchKernelGGL(k_scatter_rec, dim3(gd), dim3(256), 0, s, dd ? dd : jd, rec_d, nrec, N, nd, W.rhs);
        HELM_CHECK_LAUNCH();
        if ((rc = solve(W.w, 1)) < 0) return rc;
        for (int f = 0; f < nfreq; ++f) {
            hipLaunchKernelGGL(k_fwi_grad_freq, dim3(nb), dim3(256), 0, s, W.u + (size_t)f * nsrc * N,
                               W.w + (size_t)f * nsrc * N, (const float*)ops[f]->lv[0].g,
                               ops[f]->omega * ops[f]->omega, nsrc, N, f == 0 ? 1 : 0, W.gacc);
            HELM_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, W.gacc, N, out);
        HELM_CHECK_LAUNCH();
    }
    HELM_HIP(hipStreamSynchronize(s));
    return worst == HELM_NOT_CONVERGED ? HELM_NOT_CONVERGED : HELM_OK;
}

static int solve_opts(const helm_solve_opts* opt, const char* name, helm_solve_opts* o) {
    memset(o, 0, sizeof(*o));
    if (opt) *o = *opt;
    if (o->adjoint) return fail(HELM_EINVAL, "%s: opts.adjoint must be 0 (the call runs both solves)", name);
    o->x0_given = 0;
    return HELM_OK;
}

}  // namespace
}  // namespace helm

using namespace helm;

extern "C" int fwi_misfit_grad(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                               int nrec, const void* dobs, double tol, const helm_solve_opts* opt, double* misfit,
                               float* grad, int* iters, void* stream) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0 || !dobs || !misfit || !grad)
        return fail(HELM_EINVAL, "fwi_misfit_grad: bad arguments");
    if (!(tol > 0)) return fail(HELM_EINVAL, "fwi_misfit_grad: tol must be positive");
    int rc = check_args("fwi_misfit_grad", ops, nfreq, src_idx, nsrc, rec_idx, nrec);
    if (rc) return rc;
    helm_solve_opts o;
    if ((rc = solve_opts(opt, "fwi_misfit_grad", &o))) return rc;

    hipStream_t s = (hipStream_t)stream;
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    Owned own;
    c64* rhs = own.get<c64>((size_t)nfs * N);
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!rhs || !src_d || !rec_d) return fail(HELM_ENOMEM, "fwi_misfit_grad: workspace allocation failed");
    HELM_HIP(hipMemcpyAsync(src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemsetAsync(rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
    const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
    hipLaunchKernelGGL(k_point_sources, dim3((nfs + 255) / 256), dim3(256), 0, s, src_d, nsrc, nfs, N, amp, rhs);
    HELM_CHECK_LAUNCH();
    return misfit_grad_core(ops, nfreq, nsrc, rhs, (const c64*)dobs, rec_d, nrec, tol, o, 1.0, misfit, grad, iters, s,
                            own);
}

extern "C" int fwi_misfit_grad_encoded(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                                       const float* X, int p, const int* rec_idx, int nrec, const void* dobs,
                                       double tol, const helm_solve_opts* opt, double* misfit, float* grad,
                                       int* iters, void* stream) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !X || p <= 0 || !rec_idx || nrec <= 0 || !dobs || !misfit ||
        !grad)
        return fail(HELM_EINVAL, "fwi_misfit_grad_encoded: bad arguments");
    if (!(tol > 0)) return fail(HELM_EINVAL, "fwi_misfit_grad_encoded: tol must be positive");
    int rc = check_args("fwi_misfit_grad_encoded", ops, nfreq, src_idx, nsrc, rec_idx, nrec);
    if (rc) return rc;
    for (long q = 0; q < (long)nsrc * p; ++q)
        if (!std::isfinite(X[q])) return fail(HELM_EINVAL, "fwi_misfit_grad_encoded: X has a non-finite entry");
    helm_solve_opts o;
    if ((rc = solve_opts(opt, "fwi_misfit_grad_encoded", &o))) return rc;

    hipStream_t s = (hipStream_t)stream;
    const long N = ops[0]->n();
    const int nfp = nfreq * p;
    Owned own;
    c64* rhs = own.get<c64>((size_t)nfp * N);
    c64* dx = own.get<c64>((size_t)nfp * nrec);
    float* X_d = own.get<float>((size_t)nsrc * p);
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!rhs || !dx || !X_d || !src_d || !rec_d)
        return fail(HELM_ENOMEM, "fwi_misfit_grad_encoded: workspace allocation failed");
    HELM_HIP(hipMemcpyAsync(src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(X_d, X, sizeof(float) * (size_t)nsrc * p, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemsetAsync(rhs, 0, sizeof(c64) * (size_t)nfp * N, s));
    const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
    hipLaunchKernelGGL(k_encoded_sources, dim3((nfp + 255) / 256), dim3(256), 0, s, src_d, X_d, nsrc, p, nfp, N, amp,
                       rhs);
    HELM_CHECK_LAUNCH();
    const long total = (long)nfp * nrec;
    hipLaunchKernelGGL(k_encode_data, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const c64*)dobs, X_d,
                       nsrc, p, nrec, total, dx);
    HELM_CHECK_LAUNCH();
    return misfit_grad_core(ops, nfreq, p, rhs, dx, rec_d, nrec, tol, o, 1.0 / p, misfit, grad, iters, s, own);
}

// Shared set-up of the three linearised entry points.
static int born_entry(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                      const int* rec_idx, int nrec, const float* dm, const void* dd, void* jdm, float* out, double tol,
                      const helm_solve_opts* opt, int* iters, void* stream) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec);
    if (rc) return rc;
    helm_solve_opts o;
    if ((rc = solve_opts(opt, name, &o))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!src_d || !rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemcpyAsync(src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    BornWork W;
    if ((rc = born_alloc(own, ops[0]->n(), nfreq * nsrc, (long)nfreq * nsrc * nrec, W))) return rc;
    return born_core(ops, nfreq, nsrc, src_d, rec_d, nrec, dm, (const c64*)dd, (c64*)jdm, out, tol, o, iters, s, W,
                     false);
}

extern "C" int fwi_born(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                        const float* dm, double tol, const helm_solve_opts* opt, void* jdm, int* iters,
                        void* stream) {
    if (!dm || !jdm) return fail(HELM_EINVAL, "fwi_born: bad arguments");
    return born_entry("fwi_born", ops, nfreq, src_idx, nsrc, rec_idx, nrec, dm, nullptr, jdm, nullptr, tol, opt, iters,
                      stream);
}

extern "C" int fwi_born_adjoint(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                                int nrec, const void* dd, double tol, const helm_solve_opts* opt, float* out,
                                int* iters, void* stream) {
    if (!dd || !out) return fail(HELM_EINVAL, "fwi_born_adjoint: bad arguments");
    return born_entry("fwi_born_adjoint", ops, nfreq, src_idx, nsrc, rec_idx, nrec, nullptr, dd, nullptr, out, tol,
                      opt, iters, stream);
}

extern "C" int fwi_gn_hessvec(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                              int nrec, const float* dm, double tol, const helm_solve_opts* opt, float* out,
                              int* iters, void* stream) {
    if (!dm || !out) return fail(HELM_EINVAL, "fwi_gn_hessvec: bad arguments");
    return born_entry("fwi_gn_hessvec", ops, nfreq, src_idx, nsrc, rec_idx, nrec, dm, nullptr, nullptr, out, tol, opt,
                      iters, stream);
}

// cg_iters CG steps from x = 0 on (Re(J^H J) + damping I) x = sign * b (b float
// [N], device) into x_out (float, device); FP64 vector work, dot products
// folded in a fixed order; the point-source fields are computed on the first
// product and reused.
static int gn_cg_core(const char* name, const helm_op_t* ops, int nfreq, int nsrc, const int* src_d, const int* rec_d,
                      int nrec, const float* b, double sign, double damping, int cg_iters, double tol,
                      const helm_solve_opts& o, float* x_out, double* resnorms, hipStream_t s, Owned& own,
                      const BornWork* fields = nullptr) {
    const long N = ops[0]->n();
    double* x = own.get<double>(N);
    double* r = own.get<double>(N);
    double* p = own.get<double>(N);
    double* ap = own.get<double>(N);
    float* pf = own.get<float>(N);
    float* hp = own.get<float>(N);
    double* part = own.get<double>(CG_BLOCKS);
    if (!x || !r || !p || !ap || !pf || !hp || !part) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    BornWork W;
    int rc;
    if (fields)
        W = *fields;   // the point-source fields are already in W.u
    else if ((rc = born_alloc(own, N, nfreq * nsrc, (long)nfreq * nsrc * nrec, W)))
        return rc;
    std::vector<double> hpart(CG_BLOCKS);
    auto dot = [&](const double* a, const double* c, double* result) -> int {
        hipLaunchKernelGGL(k_cg_dot, dim3(CG_BLOCKS), dim3(256), 0, s, a, c, N, part);
        HELM_CHECK_LAUNCH();
        HELM_HIP(hipMemcpyAsync(hpart.data(), part, sizeof(double) * CG_BLOCKS, hipMemcpyDeviceToHost, s));
        HELM_HIP(hipStreamSynchronize(s));
        double acc = 0;
        for (int i = 0; i < CG_BLOCKS; ++i) acc += hpart[i];
        *result = acc;
        return HELM_OK;
    };
    const unsigned nb = (unsigned)((N + 255) / 256);
    HELM_HIP(hipMemsetAsync(x, 0, sizeof(double) * N, s));
    hipLaunchKernelGGL(k_f2d_scaled, dim3(nb), dim3(256), 0, s, b, sign, N, r);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipMemcpyAsync(p, r, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    double rr;
    if ((rc = dot(r, r, &rr))) return rc;
    if (resnorms) resnorms[0] = std::sqrt(rr);
    int worst = HELM_OK;
    for (int k = 0; k < cg_iters; ++k) {
        if (rr == 0) {   // b = 0 or an exact solution: the remaining steps change nothing
            if (resnorms)
                for (int q = k + 1; q <= cg_iters; ++q) resnorms[q] = 0;
            break;
        }
        hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, p, N, pf);
        HELM_CHECK_LAUNCH();
        rc = born_core(ops, nfreq, nsrc, src_d, rec_d, nrec, pf, nullptr, nullptr, hp, tol, o, nullptr, s, W,
                       fields != nullptr || k > 0);
        if (rc < 0) return rc;
        worst = std::max(worst, rc);
        hipLaunchKernelGGL(k_cg_ap, dim3(nb), dim3(256), 0, s, hp, p, damping, N, ap);
        HELM_CHECK_LAUNCH();
        double pap;
        if ((rc = dot(p, ap, &pap))) return rc;
        if (!(pap > 0)) return fail(HELM_ENAN, "%s: p.Ap = %g at step %d (the system is not positive definite)",
                                    name, pap, k);
        const double alpha = rr / pap;
        hipLaunchKernelGGL(k_cg_xr, dim3(nb), dim3(256), 0, s, x, r, p, ap, alpha, N);
        HELM_CHECK_LAUNCH();
        double rr_new;
        if ((rc = dot(r, r, &rr_new))) return rc;
        if (resnorms) resnorms[k + 1] = std::sqrt(rr_new);
        hipLaunchKernelGGL(k_cg_p, dim3(nb), dim3(256), 0, s, p, r, rr_new / rr, N);
        HELM_CHECK_LAUNCH();
        rr = rr_new;
    }
    hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, x, N, x_out);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipStreamSynchronize(s));
    return worst == HELM_NOT_CONVERGED ? HELM_NOT_CONVERGED : HELM_OK;
}

// Shared argument checks and source/receiver upload of the Gauss-Newton entry points.
static int gn_setup(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                    const int* rec_idx, int nrec, double damping, int cg_iters, double tol, const helm_solve_opts* opt,
                    helm_solve_opts* o, int** src_d, int** rec_d, hipStream_t s, Owned& own) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0 || cg_iters < 0)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(damping >= 0) || !std::isfinite(damping)) return fail(HELM_EINVAL, "%s: damping must be >= 0", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec);
    if (rc) return rc;
    if ((rc = solve_opts(opt, name, o))) return rc;
    *src_d = own.get<int>(nsrc);
    *rec_d = own.get<int>(nrec);
    if (!*src_d || !*rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemcpyAsync(*src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(*rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    return HELM_OK;
}

extern "C" int fwi_gn_cg(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                         const float* b, double damping, int cg_iters, double tol, const helm_solve_opts* opt,
                         float* x_out, double* resnorms, void* stream) {
    const char* name = "fwi_gn_cg";
    if (!b || !x_out) return fail(HELM_EINVAL, "%s: bad arguments", name);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    helm_solve_opts o;
    int *src_d = nullptr, *rec_d = nullptr;
    int rc = gn_setup(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, damping, cg_iters, tol, opt, &o, &src_d, &rec_d,
                      s, own);
    if (rc) return rc;
    return gn_cg_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, b, 1.0, damping, cg_iters, tol, o, x_out, resnorms,
                      s, own);
}

extern "C" int fwi_gn_step(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                           int nrec, const void* dobs, const float* m, double damping, int cg_iters, double mu,
                           double tol, const helm_solve_opts* opt, float* m_new, double* misfit, float* grad,
                           double* resnorms, void* stream) {
    const char* name = "fwi_gn_step";
    if (!dobs || !m || !m_new || !misfit || !grad || !std::isfinite(mu))
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    helm_solve_opts o;
    int *src_d = nullptr, *rec_d = nullptr;
    int rc = gn_setup(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, damping, cg_iters, tol, opt, &o, &src_d, &rec_d,
                      s, own);
    if (rc) return rc;
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    // misfit and gradient at m (the operators' model)
    BornWork W;
    if ((rc = born_alloc(own, N, nfs, (long)nfs * nrec, W))) return rc;
    float* dm = own.get<float>(N);
    if (!dm) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemsetAsync(W.rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
    const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
    hipLaunchKernelGGL(k_point_sources, dim3((nfs + 255) / 256), dim3(256), 0, s, src_d, nsrc, nfs, N, amp, W.rhs);
    HELM_CHECK_LAUNCH();
    // the gradient's forward solves leave the point-source fields in W.u for the CG
    rc = misfit_grad_core(ops, nfreq, nsrc, W.rhs, (const c64*)dobs, rec_d, nrec, tol, o, 1.0, misfit, grad, nullptr,
                          s, own, W.u);
    if (rc < 0) return rc;
    int worst = rc;
    // dm from CG on -grad, then m_new = m + mu dm
    rc = gn_cg_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, grad, -1.0, damping, cg_iters, tol, o, dm, resnorms, s,
                    own, &W);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    hipLaunchKernelGGL(k_model_update, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, m, dm, mu, N, m_new);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipStreamSynchronize(s));
    return worst == HELM_NOT_CONVERGED ? HELM_NOT_CONVERGED : HELM_OK;
}
