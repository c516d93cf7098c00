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
// Gauss-Newton (Sec. 3.3, eq. 3.9-3.11): products with J and J^H, conjugate
// gradients on (Re(J^H J) + alpha nabla^2 R + damping I) dm = -grad, and one
// step m + mu dm, with the regularisers R_high and R_diff of eq. 5.1 and 5.2.
//
// Simultaneous sources (Sec. 3.2, eq. 3.6-3.8): with an ns x p matrix X of
// Rademacher columns (drawn by the caller), the frequency's source sum is
// replaced by the trace estimate (1/p) sum_i || R H_f^{-1} G x_i - D_f x_i ||^2:
// p encoded sources G x_i and encoded data D_f x_i take the place of the ns
// point sources and their data, and misfit and gradient carry the factor 1/p.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
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

// ------------------------------------------------------------------ regularisers (eq. 5.1, 5.2)
// R_high = ||Lap_h (m - m_ref)||^2 and R_diff = ||grad_h (m - m_ref)||^2 with
// grad_h the forward differences between neighbouring nodes and
// Lap_h = -grad_h^T grad_h (each node sums (d_nb - d) / h^2 over the
// neighbours that exist).  Gradients 2 Lap_h^2 d and -2 Lap_h d, Hessians
// 2 Lap_h^2 and -2 Lap_h; all FP64.

// d = m - m_ref (FP64)
__global__ void k_model_diff(const float* __restrict__ m, const float* __restrict__ mref, long n,
                             double* __restrict__ d) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) d[t] = (double)m[t] - (double)mref[t];
}

// out = Lap_h d (nodal-gradient closure)
__global__ void k_reg_lap(const double* __restrict__ d, int nz, int nx, double ax, double az,
                          double* __restrict__ out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nz * nx) return;
    const int i = (int)(t / nx), k = (int)(t - (long)i * nx);
    const double c = d[t];
    double acc = 0;
    if (k > 0) acc += ax * (d[t - 1] - c);
    if (k + 1 < nx) acc += ax * (d[t + 1] - c);
    if (i > 0) acc += az * (d[t - nx] - c);
    if (i + 1 < nz) acc += az * (d[t + nx] - c);
    out[t] = acc;
}

// y += a x
__global__ void k_axpy_d(double* __restrict__ y, const double* __restrict__ x, double a, long n) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

// Number of entries where a and b differ (bit patterns), one atomic per wave that sees one.
__global__ void k_count_diff(const float* __restrict__ a, const float* __restrict__ b, long n, int* __restrict__ cnt) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool d = t < n && __float_as_uint(a[t]) != __float_as_uint(b[t]);
    if (__any(d) && (threadIdx.x & 63) == 0) atomicAdd(cnt, 1);
}

// ------------------------------------------------------------------ workspace
// Device workspace of the FWI entry points, grown on demand and kept for the
// next call: a call on the 512 x 512, 4-frequency, 128-source setting needs
// several GB, and the Gauss-Newton driver calls these entry points once per
// step.  A call takes the pool's slots in order; calls are serialised by
// g_fwi_mutex, and every entry point synchronises its stream before it
// returns, so a slot is never in use when the next call takes it.
struct Pool {
    std::vector<std::pair<void*, size_t>> slot;
    size_t next = 0;
    void release() {
        for (auto& sl : slot)
            if (sl.first) (void)hipFree(sl.first);
        slot.clear();
        next = 0;
    }
};
static Pool g_pool;
static std::recursive_mutex g_fwi_mutex;

struct Owned {
    Owned() { g_pool.next = 0; }
    template <typename T>
    T* get(size_t n) {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        if (g_pool.next == g_pool.slot.size()) g_pool.slot.push_back({nullptr, 0});
        auto& sl = g_pool.slot[g_pool.next++];
        if (sl.second < bytes) {
            if (sl.first) (void)hipFree(sl.first);
            sl = {nullptr, 0};
            if (hipMalloc(&sl.first, bytes) != hipSuccess) {
                sl.first = nullptr;
                return nullptr;
            }
            sl.second = bytes;
        }
        return (T*)sl.first;
    }
};

// Checks shared by the entry points: one grid, in-range sources, distinct
// in-range receivers, and one medium (every operator's m and gamma equal to
// ops[0]'s, and to m when it is given: the gradient and the model update refer
// to that one model).
static int check_args(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                      const int* rec_idx, int nrec, hipStream_t s, Owned& own, const float* m = nullptr) {
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
    const int ncmp = 2 * (nfreq - 1) + (m ? 1 : 0);
    if (ncmp == 0) return HELM_OK;
    int* cnt = own.get<int>(ncmp);
    if (!cnt) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * ncmp, s));
    const unsigned nb = (unsigned)((N + 255) / 256);
    for (int f = 1; f < nfreq; ++f) {
        hipLaunchKernelGGL(k_count_diff, dim3(nb), dim3(256), 0, s, ops[f]->lv[0].k2, ops[0]->lv[0].k2, N,
                           cnt + 2 * (f - 1));
        hipLaunchKernelGGL(k_count_diff, dim3(nb), dim3(256), 0, s, ops[f]->lv[0].g, ops[0]->lv[0].g, N,
                           cnt + 2 * (f - 1) + 1);
    }
    if (m) hipLaunchKernelGGL(k_count_diff, dim3(nb), dim3(256), 0, s, m, ops[0]->lv[0].k2, N, cnt + ncmp - 1);
    HELM_CHECK_LAUNCH();
    std::vector<int> h(ncmp);
    HELM_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int) * ncmp, hipMemcpyDeviceToHost, s));
    HELM_HIP(hipStreamSynchronize(s));
    for (int f = 1; f < nfreq; ++f)
        if (h[2 * (f - 1)] || h[2 * (f - 1) + 1])
            return fail(HELM_EINVAL, "%s: operator %d was set up with another model or attenuation than operator 0",
                        name, f);
    if (m && h[ncmp - 1]) return fail(HELM_EINVAL, "%s: m is not the model the operators were set up with", name);
    return HELM_OK;
}

// One batched solve inside an FWI entry point: the per-RHS HELM_ENAN that
// helm_solve reports as a soft failure is a hard error here (a non-finite
// field would enter the misfit, gradient or model update).
static int fwi_solve(const char* name, const helm_op_t* ops, int nfreq, const std::vector<int>& rhs_op,
                     const c64* rhs, c128* x, double tol, const helm_solve_opts& o, int* it, hipStream_t s) {
    const int nfs = (int)rhs_op.size();
    std::vector<int> st(nfs);
    const int rc = helm_solve(ops, nfreq, rhs_op.data(), rhs, x, nfs, tol, &o, it, nullptr, st.data(), s);
    if (rc < 0) return rc;
    for (int i = 0; i < nfs; ++i)
        if (st[i] == HELM_ENAN)
            return fail(HELM_ENAN, "%s: solve %d (frequency %d) produced a non-finite residual", name, i,
                        rhs_op[i]);
    return rc;
}

// From nper prepared right-hand sides per frequency (rhs, zero outside the
// sources) and their data dobs_d [nfreq][nper][nrec] (device): forward solves,
// residuals and misfit, adjoint solves, gradient; misfit and gradient times
// scale, plus extra (device FP64 [N], may be NULL) added to the gradient before
// it is rounded to float.  u_keep / lam_buf: caller-owned field buffers
// (nfreq * nper c128 fields each), else taken from the workspace.
static int misfit_grad_core(const char* name, const helm_op_t* ops, int nfreq, int nper, c64* rhs,
                            const c64* dobs_d, const int* rec_d, int nrec, double tol, helm_solve_opts o,
                            double scale, double* misfit, float* grad, int* iters, hipStream_t s, Owned& own,
                            c128* u_keep = nullptr, c128* lam_buf = nullptr, const double* extra = nullptr) {
    const long N = ops[0]->n();
    const int nfs = nfreq * nper;
    c128* u = u_keep ? u_keep : own.get<c128>((size_t)nfs * N);
    c128* lam = lam_buf ? lam_buf : own.get<c128>((size_t)nfs * N);
    double* gacc = own.get<double>(N);
    double* part = own.get<double>(nfs);
    if (!u || !lam || !gacc || !part) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    std::vector<int> rhs_op(nfs);
    for (int i = 0; i < nfs; ++i) rhs_op[i] = i / nper;
    std::vector<int> it(nfs);

    // forward solves
    o.adjoint = 0;
    int rc = fwi_solve(name, ops, nfreq, rhs_op, rhs, u, tol, o, it.data(), s);
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
    rc = fwi_solve(name, ops, nfreq, rhs_op, rhs, lam, tol, o, it.data(), s);
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
    if (extra) {
        hipLaunchKernelGGL(k_axpy_d, dim3(nb), dim3(256), 0, s, gacc, extra, 1.0, N);
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

static int born_alloc(const char* name, Owned& own, long N, int nfs, long nd, BornWork& W) {
    W.rhs = own.get<c64>((size_t)nfs * N);
    W.u = own.get<c128>((size_t)nfs * N);
    W.w = own.get<c128>((size_t)nfs * N);
    W.jd = own.get<c64>((size_t)nd);
    W.gacc = own.get<double>(N);
    if (!W.rhs || !W.u || !W.w || !W.jd || !W.gacc) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    return HELM_OK;
}

// Linearised data and its adjoint (eq. 3.10, with the sign derived from
// eq. 3.1): from the point-source fields u_fs (computed into W.u at tol_fwd
// unless have_u),
//   J dm      = R H_f^{-1} (w_f^2 (1 - i gamma) u_fs dm)          (when dm != NULL)
//   Re(J^H d) = sum_fs w_f^2 Re(conj(H_f^{-*} R^T d_fs) (1 - i gamma) u_fs)
// with d = dd, or d = J dm when dd is NULL (the Gauss-Newton product); the
// Born and adjoint solves run at tol_lin.  jdm (device c64
// [nfreq][nsrc][nrec], may be NULL) receives J dm, out (device float [nz][nx],
// may be NULL) Re(J^H d); iters receives one [nfreq][nsrc] block per solve
// batch in the order forward, Born, adjoint.
static int born_core(const char* name, const helm_op_t* ops, int nfreq, int nsrc, const int* src_d,
                     const int* rec_d, int nrec, const float* dm, const c64* dd, c64* jdm, float* out, double tol_fwd,
                     double tol_lin, helm_solve_opts o, int* iters, hipStream_t s, const BornWork& W, bool have_u) {
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    const long nd = (long)nfs * nrec;
    c64* jd = jdm ? jdm : W.jd;
    std::vector<int> rhs_op(nfs);
    for (int i = 0; i < nfs; ++i) rhs_op[i] = i / nsrc;
    std::vector<int> it(nfs);
    int worst = HELM_OK, stage = 0;
    auto solve = [&](c128* x, int adjoint, double tol) {
        o.adjoint = adjoint;
        const int rc = fwi_solve(name, ops, nfreq, rhs_op, W.rhs, x, tol, o, it.data(), s);
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
        if ((rc = solve(W.u, 0, tol_fwd)) < 0) return rc;
    }

    // J dm
    if (dm) {
        for (int f = 0; f < nfreq; ++f) {
            hipLaunchKernelGGL(k_born_source, dim3(nb), dim3(256), 0, s, W.u + (size_t)f * nsrc * N,
                               (const float*)ops[f]->lv[0].g, dm, ops[f]->omega * ops[f]->omega, nsrc, N,
                               W.rhs + (size_t)f * nsrc * N);
            HELM_CHECK_LAUNCH();
        }
        if ((rc = solve(W.w, 0, tol_lin)) < 0) return rc;
        hipLaunchKernelGGL(k_sample_rec, dim3(gd), dim3(256), 0, s, W.w, rec_d, nrec, N, nd, jd);
        HELM_CHECK_LAUNCH();
    }

    // Re(J^H d)
    if (out) {
        HELM_HIP(hipMemsetAsync(W.rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
        hipLaunchKernelGGL(k_scatter_rec, dim3(gd), dim3(256), 0, s, dd ? dd : jd, rec_d, nrec, N, nd, W.rhs);
        HELM_CHECK_LAUNCH();
        if ((rc = solve(W.w, 1, tol_lin)) < 0) return rc;
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

// Deterministic FP64 dot product: fixed blocks, partials added on the host in order.
static int dot_d(const double* a, const double* b, long n, double* part, double* result, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dot, dim3(CG_BLOCKS), dim3(256), 0, s, a, b, n, part);
    HELM_CHECK_LAUNCH();
    double hp[CG_BLOCKS];
    HELM_HIP(hipMemcpyAsync(hp, part, sizeof(double) * CG_BLOCKS, hipMemcpyDeviceToHost, s));
    HELM_HIP(hipStreamSynchronize(s));
    double acc = 0;
    for (int i = 0; i < CG_BLOCKS; ++i) acc += hp[i];
    *result = acc;
    return HELM_OK;
}

// Regulariser terms around d: out = coef * (Hessian of R) v for v (device FP64
// [N]), added to out (FP64): R_high: 2 Lap^2 v, R_diff: -2 Lap v.  tmp, tmp2: [N].
static int reg_hess_add(const helm_op* op, int kind, double coef, const double* v, double* out, double* tmp,
                        double* tmp2, hipStream_t s) {
    const long N = op->n();
    const unsigned nb = (unsigned)((N + 255) / 256);
    const double ax = 1.0 / (op->hx * op->hx), az = 1.0 / (op->hz * op->hz);
    hipLaunchKernelGGL(k_reg_lap, dim3(nb), dim3(256), 0, s, v, op->nz, op->nx, ax, az, tmp);
    HELM_CHECK_LAUNCH();
    if (kind == FWI_REG_HIGH) {
        hipLaunchKernelGGL(k_reg_lap, dim3(nb), dim3(256), 0, s, tmp, op->nz, op->nx, ax, az, tmp2);
        HELM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_axpy_d, dim3(nb), dim3(256), 0, s, out, tmp2, 2.0 * coef, N);
    } else {
        hipLaunchKernelGGL(k_axpy_d, dim3(nb), dim3(256), 0, s, out, tmp, -2.0 * coef, N);
    }
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

// Gauss-Newton options with the defaults filled in and checked.
static int gn_opts(const char* name, const fwi_gn_opts* g, double tol, const helm_op* op0, fwi_gn_opts* out) {
    if (!g) return fail(HELM_EINVAL, "%s: NULL options", name);
    *out = *g;
    if (!(out->damping >= 0) || !std::isfinite(out->damping)) return fail(HELM_EINVAL, "%s: damping must be >= 0", name);
    if (out->cg_iters < 0) return fail(HELM_EINVAL, "%s: cg_iters must be >= 0", name);
    if (!(out->tol_sens > 0)) out->tol_sens = tol;
    if (out->reg < FWI_REG_NONE || out->reg > FWI_REG_DIFF) return fail(HELM_EINVAL, "%s: unknown regulariser", name);
    if (out->reg != FWI_REG_NONE) {
        if (!(out->alpha >= 0) || !std::isfinite(out->alpha)) return fail(HELM_EINVAL, "%s: alpha must be >= 0", name);
        if (!out->m_ref) return fail(HELM_EINVAL, "%s: the regulariser needs m_ref", name);
    }
    (void)op0;
    return HELM_OK;
}

// cg_iters CG steps from x = 0 on (Re(J^H J) + alpha nabla^2 R + damping I) x =
// sign * b (b float [N], device) into x_out (float, device); FP64 vector work,
// dot products folded in a fixed order; the point-source fields are computed
// on the first product (at tol) and reused; the Born and adjoint solves run at
// g.tol_sens.  iters (host, may be NULL): [cg_iters][2][nfreq][nsrc], Born then
// adjoint batch of each step (0 after an early stop).
static int gn_cg_core(const char* name, const helm_op_t* ops, int nfreq, int nsrc, const int* src_d, const int* rec_d,
                      int nrec, const float* b, double sign, const fwi_gn_opts& g, double tol,
                      const helm_solve_opts& o, float* x_out, double* resnorms, int* iters, hipStream_t s, Owned& own,
                      const BornWork* fields = nullptr) {
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    double* x = own.get<double>(N);
    double* r = own.get<double>(N);
    double* p = own.get<double>(N);
    double* ap = own.get<double>(N);
    double* t1 = own.get<double>(N);
    double* t2 = own.get<double>(N);
    float* pf = own.get<float>(N);
    float* hp = own.get<float>(N);
    double* part = own.get<double>(CG_BLOCKS);
    if (!x || !r || !p || !ap || !t1 || !t2 || !pf || !hp || !part)
        return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    BornWork W;
    int rc;
    if (fields)
        W = *fields;   // the point-source fields are already in W.u
    else if ((rc = born_alloc(name, own, N, nfs, (long)nfs * nrec, W)))
        return rc;
    if (iters) std::fill(iters, iters + (size_t)g.cg_iters * 2 * nfs, 0);
    const unsigned nb = (unsigned)((N + 255) / 256);
    HELM_HIP(hipMemsetAsync(x, 0, sizeof(double) * N, s));
    hipLaunchKernelGGL(k_f2d_scaled, dim3(nb), dim3(256), 0, s, b, sign, N, r);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipMemcpyAsync(p, r, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    double rr;
    if ((rc = dot_d(r, r, N, part, &rr, s))) return rc;
    if (resnorms) resnorms[0] = std::sqrt(rr);
    int worst = HELM_OK;
    std::vector<int> it3(3 * (size_t)nfs);
    for (int k = 0; k < g.cg_iters; ++k) {
        if (rr == 0) {   // b = 0 or an exact solution: the remaining steps change nothing
            if (resnorms)
                for (int q = k + 1; q <= g.cg_iters; ++q) resnorms[q] = 0;
            break;
        }
        hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, p, N, pf);
        HELM_CHECK_LAUNCH();
        const bool have_u = fields != nullptr || k > 0;
        rc = born_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, pf, nullptr, nullptr, hp, tol, g.tol_sens, o,
                       iters ? it3.data() : nullptr, s, W, have_u);
        if (rc < 0) return rc;
        worst = std::max(worst, rc);
        if (iters) {
            // born_core's batches: [forward,] Born, adjoint
            const int* src = it3.data() + (have_u ? 0 : nfs);
            std::copy(src, src + 2 * (size_t)nfs, iters + (size_t)k * 2 * nfs);
        }
        hipLaunchKernelGGL(k_cg_ap, dim3(nb), dim3(256), 0, s, hp, p, g.damping, N, ap);
        HELM_CHECK_LAUNCH();
        if (g.reg != FWI_REG_NONE && g.alpha > 0 &&
            (rc = reg_hess_add(ops[0], g.reg, g.alpha, p, ap, t1, t2, s)))
            return rc;
        double pap;
        if ((rc = dot_d(p, ap, N, part, &pap, s))) return rc;
        if (!(pap > 0)) return fail(HELM_ENAN, "%s: p.Ap = %g at step %d (the system is not positive definite)",
                                    name, pap, k);
        const double step = rr / pap;
        hipLaunchKernelGGL(k_cg_xr, dim3(nb), dim3(256), 0, s, x, r, p, ap, step, N);
        HELM_CHECK_LAUNCH();
        double rr_new;
        if ((rc = dot_d(r, r, N, part, &rr_new, s))) return rc;
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

}  // namespace
}  // namespace helm

using namespace helm;

extern "C" int fwi_misfit_grad(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                               int nrec, const void* dobs, double tol, const helm_solve_opts* opt, double* misfit,
                               float* grad, int* iters, void* stream) {
    const char* name = "fwi_misfit_grad";
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0 || !dobs || !misfit || !grad)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, s, own);
    if (rc) return rc;
    helm_solve_opts o;
    if ((rc = solve_opts(opt, name, &o))) return rc;

    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    c64* rhs = own.get<c64>((size_t)nfs * N);
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!rhs || !src_d || !rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemcpyAsync(src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemsetAsync(rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
    const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
    hipLaunchKernelGGL(k_point_sources, dim3((nfs + 255) / 256), dim3(256), 0, s, src_d, nsrc, nfs, N, amp, rhs);
    HELM_CHECK_LAUNCH();
    return misfit_grad_core(name, ops, nfreq, nsrc, rhs, (const c64*)dobs, rec_d, nrec, tol, o, 1.0, misfit, grad,
                            iters, s, own);
}

extern "C" int fwi_misfit_grad_encoded(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                                       const float* X, int p, const int* rec_idx, int nrec, const void* dobs,
                                       double tol, const helm_solve_opts* opt, double* misfit, float* grad,
                                       int* iters, void* stream) {
    const char* name = "fwi_misfit_grad_encoded";
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !X || p <= 0 || !rec_idx || nrec <= 0 || !dobs || !misfit ||
        !grad)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    for (long q = 0; q < (long)nsrc * p; ++q)
        if (!std::isfinite(X[q])) return fail(HELM_EINVAL, "%s: X has a non-finite entry", name);
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, s, own);
    if (rc) return rc;
    helm_solve_opts o;
    if ((rc = solve_opts(opt, name, &o))) return rc;

    const long N = ops[0]->n();
    const int nfp = nfreq * p;
    c64* rhs = own.get<c64>((size_t)nfp * N);
    c64* dx = own.get<c64>((size_t)nfp * nrec);
    float* X_d = own.get<float>((size_t)nsrc * p);
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!rhs || !dx || !X_d || !src_d || !rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
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
    return misfit_grad_core(name, ops, nfreq, p, rhs, dx, rec_d, nrec, tol, o, 1.0 / p, misfit, grad, iters, s, own);
}

// Shared set-up of the three linearised entry points.
static int born_entry(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                      const int* rec_idx, int nrec, const float* dm, const void* dd, void* jdm, float* out, double tol,
                      const helm_solve_opts* opt, int* iters, void* stream) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, s, own);
    if (rc) return rc;
    helm_solve_opts o;
    if ((rc = solve_opts(opt, name, &o))) return rc;
    int* src_d = own.get<int>(nsrc);
    int* rec_d = own.get<int>(nrec);
    if (!src_d || !rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemcpyAsync(src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    BornWork W;
    if ((rc = born_alloc(name, own, ops[0]->n(), nfreq * nsrc, (long)nfreq * nsrc * nrec, W))) return rc;
    return born_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, dm, (const c64*)dd, (c64*)jdm, out, tol, tol, o,
                     iters, s, W, false);
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

// Shared argument checks and source/receiver upload of the Gauss-Newton entry points.
static int gn_setup(const char* name, const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc,
                    const int* rec_idx, int nrec, const fwi_gn_opts* gopt, double tol, const helm_solve_opts* opt,
                    fwi_gn_opts* g, helm_solve_opts* o, int** src_d, int** rec_d, hipStream_t s, Owned& own,
                    const float* m = nullptr) {
    if (!ops || nfreq <= 0 || !src_idx || nsrc <= 0 || !rec_idx || nrec <= 0)
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    if (!(tol > 0)) return fail(HELM_EINVAL, "%s: tol must be positive", name);
    int rc = check_args(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, s, own, m);
    if (rc) return rc;
    if ((rc = gn_opts(name, gopt, tol, ops[0], g))) return rc;
    if ((rc = solve_opts(opt, name, o))) return rc;
    *src_d = own.get<int>(nsrc);
    *rec_d = own.get<int>(nrec);
    if (!*src_d || !*rec_d) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    HELM_HIP(hipMemcpyAsync(*src_d, src_idx, sizeof(int) * nsrc, hipMemcpyHostToDevice, s));
    HELM_HIP(hipMemcpyAsync(*rec_d, rec_idx, sizeof(int) * nrec, hipMemcpyHostToDevice, s));
    return HELM_OK;
}

extern "C" int fwi_gn_cg(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                         const float* b, const fwi_gn_opts* gopt, double tol, const helm_solve_opts* opt,
                         float* x_out, double* resnorms, int* iters, void* stream) {
    const char* name = "fwi_gn_cg";
    if (!b || !x_out) return fail(HELM_EINVAL, "%s: bad arguments", name);
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    fwi_gn_opts g;
    helm_solve_opts o;
    int *src_d = nullptr, *rec_d = nullptr;
    int rc = gn_setup(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, gopt, tol, opt, &g, &o, &src_d, &rec_d, s, own);
    if (rc) return rc;
    return gn_cg_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, b, 1.0, g, tol, o, x_out, resnorms, iters, s, own);
}

extern "C" int fwi_gn_step(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx,
                           int nrec, const void* dobs, const float* m, const fwi_gn_opts* gopt, double mu, double tol,
                           const helm_solve_opts* opt, float* m_new, double* misfit, double* reg_value, float* grad,
                           double* resnorms, int* iters, void* stream) {
    const char* name = "fwi_gn_step";
    if (!dobs || !m || !m_new || !misfit || !grad || !std::isfinite(mu))
        return fail(HELM_EINVAL, "%s: bad arguments", name);
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    hipStream_t s = (hipStream_t)stream;
    Owned own;
    fwi_gn_opts g;
    helm_solve_opts o;
    int *src_d = nullptr, *rec_d = nullptr;
    int rc = gn_setup(name, ops, nfreq, src_idx, nsrc, rec_idx, nrec, gopt, tol, opt, &g, &o, &src_d, &rec_d, s, own,
                      m);
    if (rc) return rc;
    const long N = ops[0]->n();
    const int nfs = nfreq * nsrc;
    const unsigned nb = (unsigned)((N + 255) / 256);
    BornWork W;
    if ((rc = born_alloc(name, own, N, nfs, (long)nfs * nrec, W))) return rc;
    float* dm = own.get<float>(N);
    double* regg = own.get<double>(N);
    double* d = own.get<double>(N);
    double* t = own.get<double>(N);
    double* part = own.get<double>(CG_BLOCKS);
    if (!dm || !regg || !d || !t || !part) return fail(HELM_ENOMEM, "%s: workspace allocation failed", name);
    // regulariser value and alpha dR/dm at m (FP64), added to the data gradient
    double rv = 0;
    const bool reg = g.reg != FWI_REG_NONE;
    if (reg) {
        hipLaunchKernelGGL(k_model_diff, dim3(nb), dim3(256), 0, s, m, g.m_ref, N, d);
        HELM_CHECK_LAUNCH();
        const double ax = 1.0 / (ops[0]->hx * ops[0]->hx), az = 1.0 / (ops[0]->hz * ops[0]->hz);
        hipLaunchKernelGGL(k_reg_lap, dim3(nb), dim3(256), 0, s, d, ops[0]->nz, ops[0]->nx, ax, az, t);
        HELM_CHECK_LAUNCH();
        if (g.reg == FWI_REG_HIGH) {
            if ((rc = dot_d(t, t, N, part, &rv, s))) return rc;             // ||Lap d||^2
        } else {
            if ((rc = dot_d(d, t, N, part, &rv, s))) return rc;             // ||grad d||^2 = -d.Lap d
            rv = -rv;
        }
        HELM_HIP(hipMemsetAsync(regg, 0, sizeof(double) * N, s));
        if ((rc = reg_hess_add(ops[0], g.reg, g.alpha, d, regg, t, W.gacc, s))) return rc;   // alpha dR/dm = alpha H_R d
    }
    if (reg_value) *reg_value = rv;
    HELM_HIP(hipMemsetAsync(W.rhs, 0, sizeof(c64) * (size_t)nfs * N, s));
    const float amp = (float)(1.0 / (ops[0]->hx * ops[0]->hz));
    hipLaunchKernelGGL(k_point_sources, dim3((nfs + 255) / 256), dim3(256), 0, s, src_d, nsrc, nfs, N, amp, W.rhs);
    HELM_CHECK_LAUNCH();
    // misfit and gradient at m: the forward fields stay in W.u for the CG, the
    // adjoint fields use W.w (free until the CG needs it)
    rc = misfit_grad_core(name, ops, nfreq, nsrc, W.rhs, (const c64*)dobs, rec_d, nrec, tol, o, 1.0, misfit, grad,
                          iters, s, own, W.u, W.w, reg ? regg : nullptr);
    if (rc < 0) return rc;
    int worst = rc;
    // dm from CG on -grad, then m_new = m + mu dm
    rc = gn_cg_core(name, ops, nfreq, nsrc, src_d, rec_d, nrec, grad, -1.0, g, tol, o, dm, resnorms,
                    iters ? iters + 2 * (size_t)nfs : nullptr, s, own, &W);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
    hipLaunchKernelGGL(k_model_update, dim3(nb), dim3(256), 0, s, m, dm, mu, N, m_new);
    HELM_CHECK_LAUNCH();
    HELM_HIP(hipStreamSynchronize(s));
    return worst == HELM_NOT_CONVERGED ? HELM_NOT_CONVERGED : HELM_OK;
}

extern "C" int fwi_release_workspace(void) {
    std::lock_guard<std::recursive_mutex> lk(g_fwi_mutex);
    HELM_HIP(hipDeviceSynchronize());
    g_pool.release();
    return HELM_OK;
}
