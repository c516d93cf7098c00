// Helmholtz operator, shifted-Laplacian V-cycle and flexible-GMRES kernels for gfx950.
//
// Level-0 vector kernels use one layout: a block of 256 threads covers 512
// node pairs (1024 consecutive nodes of one right-hand side); lane t owns pairs
// t and t + 256, so each wave issues 16-byte (c64) or 32-byte (c128) loads
// that are contiguous across lanes.  blockIdx.y selects the right-hand side.
#include <cmath>

#include "internal.h"

namespace helm {

// ------------------------------------------------------------------ stencil
// H u at the node pair starting at flat index n0 (even):
//   (2u - uW - uE) ax + (2u - uN - uS) az - c u   (zero outside the grid).
template <typename T, typename U>
__device__ __forceinline__ pair2<T> stencil_pair(const cx<U>* __restrict__ u, long n0, int i, int k0, int nz, int nx,
                                                 T ax, T az, cx<T> c0, cx<T> c1) {
    const cx<T> zero = mk(T(0), T(0));
    pair2<U> cu = ld_pair(u + n0);
    cx<T> u0 = ccast<T>(cu.a), u1 = ccast<T>(cu.b);
    cx<T> w = k0 > 0 ? ccast<T>(u[n0 - 1]) : zero;
    cx<T> e = (k0 + 2 < nx) ? ccast<T>(u[n0 + 2]) : zero;
    pair2<T> nn = {zero, zero}, ss = {zero, zero};
    if (i > 0) {
        pair2<U> t = ld_pair(u + n0 - nx);
        nn = {ccast<T>(t.a), ccast<T>(t.b)};
    }
    if (i + 1 < nz) {
        pair2<U> t = ld_pair(u + n0 + nx);
        ss = {ccast<T>(t.a), ccast<T>(t.b)};
    }
    const T d = T(2) * ax + T(2) * az;
    pair2<T> r;
    r.a = d * u0 - ax * (w + u1) - az * (nn.a + ss.a) - c0 * u0;
    r.b = d * u1 - ax * (u0 + e) - az * (nn.b + ss.b) - c1 * u1;
    return r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_matvec(const cx<T>* __restrict__ coef, T ax, T az, int nz, int nx,
                                                const cx<T>* __restrict__ u, cx<T>* __restrict__ v, int conjop) {
    const long N = (long)nz * nx;
    const long base = (long)blockIdx.y * N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= N / 2) continue;
        long n0 = 2 * q;
        int i = (int)(n0 / nx), k0 = (int)(n0 - (long)i * nx);
        pair2<T> c = ld_pair(coef + n0);
        if (conjop) {
            c.a = conj(c.a);
            c.b = conj(c.b);
        }
        st_pair(v + base + n0, stencil_pair<T, T>(u + base, n0, i, k0, nz, nx, ax, az, c.a, c.b));
    }
}

template <typename T>
int launch_matvec(const helm_op* op, const cx<T>* u, cx<T>* v, int nrhs, int conj, hipStream_t s) {
    long N = op->n();
    int nblk = (int)((N / 2 + PAIRS_PER_BLOCK - 1) / PAIRS_PER_BLOCK);
    const cx<T>* coef;
    if constexpr (sizeof(T) == 4)
        coef = op->coef32;
    else
        coef = op->coef64;
    T ax = T(1.0 / (op->hx * op->hx)), az = T(1.0 / (op->hz * op->hz));
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        int nr = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        hipLaunchKernelGGL(k_matvec<T>, dim3(nblk, nr), dim3(VEC_THREADS), 0, s, coef, ax, az, op->nz, op->nx,
                           u + (long)r0 * N, v + (long)r0 * N, conj);
        HELM_CHECK_LAUNCH();
    }
    return HELM_OK;
}
template int launch_matvec<float>(const helm_op*, const c64*, c64*, int, int, hipStream_t);
template int launch_matvec<double>(const helm_op*, const c128*, c128*, int, int, hipStream_t);

// ------------------------------------------------------------------ setup (operator and hierarchy)
__global__ void k_level_coef(const float* __restrict__ k2, const float* __restrict__ g, long n, double w2,
                             double beta, int with_gamma, c64* coef32, c128* coef64, c64* sl32, c128* sl64) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double m = (double)k2[t], gg = (double)g[t];
    double a = w2 * m;
    if (coef32) {
        coef32[t] = mk((float)a, (float)(-a * gg));
        coef64[t] = mk(a, -a * gg);
    }
    double sh = (with_gamma ? gg : 0.0) + beta;
    sl32[t] = mk((float)a, (float)(-a * sh));
    sl64[t] = mk(a, -a * sh);
}

// Normalised full weighting of a real field onto the odd nodes (coarse I on fine 2I+1).
__global__ void k_restrict_field(const float* __restrict__ f, int nz, int nx, float* __restrict__ out, int cz,
                                 int cx_) {
    int J = blockIdx.x * blockDim.x + threadIdx.x;
    int I = blockIdx.y;
    if (J >= cx_ || I >= cz) return;
    const double w[3] = {0.25, 0.5, 0.25};
    double num = 0, den = 0;
    for (int a = 0; a < 3; ++a) {
        int i = 2 * I + a;
        if (i >= nz) continue;
        for (int b = 0; b < 3; ++b) {
            int k = 2 * J + b;
            if (k >= nx) continue;
            double ww = w[a] * w[b];
            num += ww * (double)f[(long)i * nx + k];
            den += ww;
        }
    }
    out[(long)I * cx_ + J] = (float)(num / den);
}

constexpr int POLY_THREADS = 1024;
constexpr int POLY_NPT = 4;
constexpr int POLY_LDS_MAX = POLY_THREADS * POLY_NPT;  // 4096 nodes, 2 x 64 KiB of LDS
template <typename T>
__global__ void k_poly_lds(const cx<T>* __restrict__ src, cx<T>* __restrict__ out, const c128* __restrict__ sl,
                           int nz, int nx, Sten<double> sten, const c128* __restrict__ roots, int deg,
                           const RhsState* __restrict__ st, int rhs0, unsigned long long* wc);

// w / D per node of a level, D = stencil diagonal (with the far-boundary rows) - mass term.
__global__ void k_level_wdinv(const c128* __restrict__ sl, int nz, int nx, Sten<double> st, double wj,
                              c64* __restrict__ wd32, c128* __restrict__ wd64) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nz * nx) return;
    int i = (int)(t / nx), k = (int)(t - (long)i * nx);
    double dg = (k == nx - 1 ? st.dxl : 2 * st.ax) + (i == nz - 1 ? st.dzl : 2 * st.az);
    c128 D = mk(dg - sl[t].re, -sl[t].im);
    c128 w = wj * cinv(D);
    wd64[t] = w;
    wd32[t] = ccast<float>(w);
}

int setup_levels(helm_op* op, const float* k2, const float* g, hipStream_t s) {
    double w2 = op->omega * op->omega;
    // the single-workgroup coarse polynomial needs 2 x 64 KiB of dynamic LDS (two residual buffers)
    static const bool lds_ok =
        hipFuncSetAttribute((const void*)k_poly_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * POLY_LDS_MAX * (int)sizeof(c128)) == hipSuccess &&
        hipFuncSetAttribute((const void*)k_poly_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * POLY_LDS_MAX * (int)sizeof(c128)) == hipSuccess;
    op->poly_lds_ok = lds_ok;
    for (int l = 0; l < op->nlev; ++l) {
        Level& L = op->lv[l];
        if (l > 0) {
            Level& F = op->lv[l - 1];
            dim3 grid((L.nx + 127) / 128, L.nz);
            hipLaunchKernelGGL(k_restrict_field, grid, dim3(128), 0, s, F.k2, F.nz, F.nx, L.k2, L.nz, L.nx);
            HELM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_restrict_field, grid, dim3(128), 0, s, F.g, F.nz, F.nx, L.g, L.nz, L.nx);
            HELM_CHECK_LAUNCH();
        }
        long n = L.n();
        hipLaunchKernelGGL(k_level_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.k2, L.g, n, w2,
                           op->beta, op->with_gamma, l == 0 ? op->coef32 : nullptr, l == 0 ? op->coef64 : nullptr,
                           L.sl32, L.sl64);
        HELM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_level_wdinv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.sl64, L.nz, L.nx,
                           L.sten<double>(), op->jw, L.wd32, L.wd64);
        HELM_CHECK_LAUNCH();
    }
    (void)k2;
    (void)g;
    return HELM_OK;
}

// ------------------------------------------------------------------ V-cycle
// The V-cycle is from e = 0 on every level, so the pre-smoothed iterate is
// e0 = w D^-1 f pointwise and never stored: the restriction kernel recomputes
// it on the fly, and the prolongation kernel recomputes it before adding the
// coarse correction and post-smoothing.
constexpr int MG_T = 16;  // coarse tile edge (restriction) / fine tile edge (prolongation)

template <typename T>
__device__ __forceinline__ cx<T> load_f(const cx<T>* __restrict__ f, long idx, T scale) {
    cx<T> v = f[idx];
    return mk(scale * v.re, scale * v.im);
}

// Level stencil pieces at node (i, k) of an nz x nx level.
template <typename T>
struct NodeSten {
    T dg, cw, ce, cn, cs;  // diagonal (without the mass term) and neighbour coefficients
};
template <typename T>
__device__ __forceinline__ NodeSten<T> node_sten(const Sten<T>& s, int i, int k, int nz, int nx) {
    NodeSten<T> r;
    const bool lx = k == nx - 1, lz = i == nz - 1;
    r.dg = (lx ? s.dxl : T(2) * s.ax) + (lz ? s.dzl : T(2) * s.az);
    r.cw = lx ? s.axl : s.ax;
    r.ce = s.ax;
    r.cn = lz ? s.azl : s.az;
    r.cs = s.az;
    return r;
}

// f (level l) -> fc = R (f - P e0) on level l+1, e0 = w D^-1 f.  Coarse node I
// sits on fine node 2I+1, so a coarse tile I0.. needs fine rows 2I0-1 .. 2I0+33.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_down(const cx<T>* __restrict__ f, const double* __restrict__ fscale,
                                                 int fstride, const cx<T>* __restrict__ wd, int nz, int nx,
                                                 Sten<T> sten, T wj, cx<T>* __restrict__ fc, int cz, int cxn,
                                                 const RhsState* __restrict__ st, int rhs0,
                                                 unsigned long long* wc) {
    const int rl = blockIdx.z;
    if (st) {
        const RhsState& S = st[rhs0 + rl];
        if (!S.active || S.cycdone) return;
    }
    const T scale = fscale ? T(fscale[(long)(rhs0 + rl) * fstride]) : T(1);
    const long N = (long)nz * nx;
    f += (long)rl * N;
    fc += (long)rl * cz * cxn;
    constexpr int P = 2 * MG_T + 3;  // fine patch edge
    __shared__ cx<T> e0s[P][P];
    __shared__ cx<T> fs[P][P];
    __shared__ cx<T> rs[P - 2][P - 2];
    const int I0 = blockIdx.y * MG_T, J0 = blockIdx.x * MG_T;
    const int fi0 = 2 * I0 - 1, fk0 = 2 * J0 - 1;
    for (int idx = threadIdx.x; idx < P * P; idx += 256) {
        int pi = idx / P, pk = idx - pi * P;
        int i = fi0 + pi, k = fk0 + pk;
        cx<T> fv = mk(T(0), T(0)), ev = mk(T(0), T(0));
        if (i >= 0 && i < nz && k >= 0 && k < nx) {
            long n = (long)i * nx + k;
            fv = load_f(f, n, scale);
            ev = wd[n] * fv;
        }
        fs[pi][pk] = fv;
        e0s[pi][pk] = ev;
    }
    __syncthreads();
    // residual f - P e0 = (1-w) f + cw eW + ce eE + cn eN + cs eS  (D e0 = w f)
    for (int idx = threadIdx.x; idx < (P - 2) * (P - 2); idx += 256) {
        int pi = idx / (P - 2) + 1, pk = idx % (P - 2) + 1;
        int i = fi0 + pi, k = fk0 + pk;
        cx<T> r = mk(T(0), T(0));
        if (i >= 0 && i < nz && k >= 0 && k < nx) {
            NodeSten<T> ns = node_sten(sten, i, k, nz, nx);
            r = (T(1) - wj) * fs[pi][pk] + ns.cw * e0s[pi][pk - 1] + ns.ce * e0s[pi][pk + 1] +
                ns.cn * e0s[pi - 1][pk] + ns.cs * e0s[pi + 1][pk];
        }
        rs[pi - 1][pk - 1] = r;
    }
    __syncthreads();
    const int ti = threadIdx.x / MG_T, tk = threadIdx.x % MG_T;
    const int I = I0 + ti, J = J0 + tk;
    {
        int tz = cz - I0 < MG_T ? cz - I0 : MG_T, tx = cxn - J0 < MG_T ? cxn - J0 : MG_T;
        add_work(wc, (unsigned long long)tz * tx * 5 * 2 * sizeof(T));
    }
    if (I < cz && J < cxn) {
        // fine node 2I + a sits at rs index 2*ti + a
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        cx<T> acc = mk(T(0), T(0));
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc = acc + (w[a] * w[b]) * rs[2 * ti + a][2 * tk + b];
        fc[(long)I * cxn + J] = acc;
    }
}

// Bilinear prolongation of the coarse correction at fine node (i, k):
// odd index -> coarse (i-1)/2, even index -> mean of coarse i/2-1 and i/2.
template <typename T>
__device__ __forceinline__ cx<T> prolong_at(const cx<T>* __restrict__ ec, int i, int k, int cz, int cxn) {
    int Ia, Ib, Ja, Jb;
    T wi, wk;
    if (i & 1) {
        Ia = (i - 1) >> 1;
        Ib = -1;
        wi = T(1);
    } else {
        Ia = (i >> 1) - 1;
        Ib = i >> 1;
        wi = T(0.5);
    }
    if (k & 1) {
        Ja = (k - 1) >> 1;
        Jb = -1;
        wk = T(1);
    } else {
        Ja = (k >> 1) - 1;
        Jb = k >> 1;
        wk = T(0.5);
    }
    cx<T> p = mk(T(0), T(0));
    const bool ja = Ja >= 0 && Ja < cxn, jb = Jb >= 0 && Jb < cxn;
    if (Ia >= 0 && Ia < cz) {
        if (ja) p = p + ec[(long)Ia * cxn + Ja];
        if (jb) p = p + ec[(long)Ia * cxn + Jb];
    }
    if (Ib >= 0 && Ib < cz) {
        if (ja) p = p + ec[(long)Ib * cxn + Ja];
        if (jb) p = p + ec[(long)Ib * cxn + Jb];
    }
    return (wi * wk) * p;
}

// out = e + w D^-1 (f - P e), e = w D^-1 f + Prol(ec)  (+ addend)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_up(const cx<T>* __restrict__ f, const double* __restrict__ fscale,
                                               int fstride, const cx<T>* __restrict__ sl,
                                               const cx<T>* __restrict__ wd, int nz, int nx,
                                               Sten<T> sten, T wj, const cx<T>* __restrict__ ec, int cz, int cxn,
                                               cx<T>* __restrict__ out, const cx<T>* __restrict__ addend,
                                               const RhsState* __restrict__ st, int rhs0, unsigned long long* wc) {
    const int rl = blockIdx.z;
    if (st) {
        const RhsState& S = st[rhs0 + rl];
        if (!S.active || S.cycdone) return;
    }
    const T scale = fscale ? T(fscale[(long)(rhs0 + rl) * fstride]) : T(1);
    const long N = (long)nz * nx;
    f += (long)rl * N;
    out += (long)rl * N;
    if (addend) addend += (long)rl * N;
    ec += (long)rl * cz * cxn;
    constexpr int P = MG_T + 2;
    __shared__ cx<T> es[P][P];
    const int i0 = blockIdx.y * MG_T - 1, k0 = blockIdx.x * MG_T - 1;
    for (int idx = threadIdx.x; idx < P * P; idx += 256) {
        int pi = idx / P, pk = idx - pi * P;
        int i = i0 + pi, k = k0 + pk;
        cx<T> ev = mk(T(0), T(0));
        if (i >= 0 && i < nz && k >= 0 && k < nx) {
            long n = (long)i * nx + k;
            ev = wd[n] * load_f(f, n, scale) + prolong_at(ec, i, k, cz, cxn);
        }
        es[pi][pk] = ev;
    }
    __syncthreads();
    const int ti = threadIdx.x / MG_T, tk = threadIdx.x % MG_T;
    const int i = i0 + 1 + ti, k = k0 + 1 + tk;
    {
        int tz = nz - (i0 + 1) < MG_T ? nz - (i0 + 1) : MG_T, tx = nx - (k0 + 1) < MG_T ? nx - (k0 + 1) : MG_T;
        // f read + out write (+ addend) per fine node, coarse correction read per coarse node
        add_work(wc, (unsigned long long)tz * tx * (addend ? 3 : 2) * 2 * sizeof(T) +
                         (unsigned long long)tz * tx / 4 * 2 * sizeof(T));
    }
    if (i < nz && k < nx) {
        long n = (long)i * nx + k;
        NodeSten<T> ns = node_sten(sten, i, k, nz, nx);
        cx<T> D = mk(ns.dg - sl[n].re, -sl[n].im);
        cx<T> e = es[ti + 1][tk + 1];
        cx<T> res = load_f(f, n, scale) - D * e + ns.cw * es[ti + 1][tk] + ns.ce * es[ti + 1][tk + 2] +
                    ns.cn * es[ti][tk + 1] + ns.cs * es[ti + 2][tk + 1];
        cx<T> o = e + wd[n] * res;
        if (addend) o = o + addend[n];
        out[n] = o;
    }
}

// One factor of the coarsest-level polynomial: x += r/theta, r' = r - P r/theta.
// Always FP64 (the product form amplifies FP32 rounding by ~1e3 on small
// coarse grids); the first factor reads the level right-hand side src (type
// T), the last writes x rounded to T into out.
template <typename T>
__global__ __launch_bounds__(256) void k_poly_term(const cx<T>* __restrict__ src, const c128* __restrict__ r,
                                                   c128* __restrict__ rn, c128* __restrict__ x,
                                                   cx<T>* __restrict__ out, const c128* __restrict__ sl, int nz,
                                                   int nx, Sten<double> sten, c128 itheta, int first, int last,
                                                   const RhsState* __restrict__ st, int rhs0,
                                                   unsigned long long* wc) {
    const int rl = blockIdx.y;
    if (st) {
        const RhsState& S = st[rhs0 + rl];
        if (!S.active || S.cycdone) return;
    }
    const long N = (long)nz * nx;
    {
        long nb = N - (long)blockIdx.x * 256;
        // r read, x written (first) or updated, next r written (not last) / output written (last)
        unsigned long long per = (first ? sizeof(cx<T>) : 16) + (first ? 16 : 32) + (last ? sizeof(cx<T>) : 16);
        add_work(wc, (unsigned long long)(nb < 256 ? nb : 256) * per);
    }
    long n = (long)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    src += (long)rl * N;
    r += (long)rl * N;
    rn += (long)rl * N;
    x += (long)rl * N;
    out += (long)rl * N;
    const int i = (int)(n / nx), k = (int)(n - (long)i * nx);
    auto val = [&](long m) -> c128 { return first ? ccast<double>(src[m]) : r[m]; };
    c128 rc = val(n);
    c128 xv = rc * itheta;
    if (!first) xv = x[n] + xv;
    if (last) {
        out[n] = ccast<T>(xv);
        return;
    }
    x[n] = xv;
    const c128 zero = mk(0.0, 0.0);
    c128 w = k > 0 ? val(n - 1) : zero, e = k + 1 < nx ? val(n + 1) : zero;
    c128 nn = i > 0 ? val(n - nx) : zero, ss = i + 1 < nz ? val(n + nx) : zero;
    NodeSten<double> ns = node_sten(sten, i, k, nz, nx);
    c128 pr = ns.dg * rc - ns.cw * w - ns.ce * e - ns.cn * nn - ns.cs * ss - sl[n] * rc;
    rn[n] = rc - pr * itheta;
}

// Whole coarsest-level polynomial in one workgroup per right-hand side, the
// residual resident in LDS (FP64) and the iterate and the diagonal terms in
// registers.  The residual is double buffered in LDS, so one barrier per
// factor suffices: a thread overwrites buffer (t+1) % 2 only after the barrier
// of factor t, which every thread reaches after its reads of factor t-1 from
// that buffer.  The factors' reciprocal roots are formed once, into LDS, at the
// start (a global load and two divisions per factor otherwise sit on every
// factor's critical path).  Used when the level has at most POLY_LDS_MAX nodes.
template <typename T>
__global__ __launch_bounds__(POLY_THREADS) void k_poly_lds(const cx<T>* __restrict__ src, cx<T>* __restrict__ out,
                                                           const c128* __restrict__ sl, int nz, int nx,
                                                           Sten<double> sten, const c128* __restrict__ roots, int deg,
                                                           const RhsState* __restrict__ st, int rhs0,
                                                           unsigned long long* wc) {
    const int rl = blockIdx.x;
    if (st) {
        const RhsState& S = st[rhs0 + rl];
        if (!S.active || S.cycdone) return;
    }
    const int N = nz * nx;
    src += (long)rl * N;
    out += (long)rl * N;
    add_work(wc, (unsigned long long)N * 2 * sizeof(cx<T>));
    extern __shared__ c128 lds_poly[];   // two residual buffers of N entries
    __shared__ c128 inv_roots[64];       // 1 / theta_t, formed once (deg <= 64)
    if (threadIdx.x < deg) {
        const c128 th = roots[threadIdx.x];
        const double d = th.re * th.re + th.im * th.im;
        inv_roots[threadIdx.x] = mk(th.re / d, -th.im / d);
    }
    c128 xr[POLY_NPT], rr[POLY_NPT], sd[POLY_NPT];
    int ii[POLY_NPT], kk[POLY_NPT];
#pragma unroll
    for (int q = 0; q < POLY_NPT; ++q) {
        int n = threadIdx.x + q * POLY_THREADS;
        xr[q] = mk(0.0, 0.0);
        rr[q] = n < N ? ccast<double>(src[n]) : mk(0.0, 0.0);
        ii[q] = n / nx;
        kk[q] = n - ii[q] * nx;
        sd[q] = mk(0.0, 0.0);
        if (n < N) {
            // stencil diagonal minus the mass term
            NodeSten<double> ns = node_sten(sten, ii[q], kk[q], nz, nx);
            sd[q] = mk(ns.dg - sl[n].re, -sl[n].im);
        }
    }
    __syncthreads();
    for (int t = 0; t < deg; ++t) {
        const c128 it = inv_roots[t];
#pragma unroll
        for (int q = 0; q < POLY_NPT; ++q) xr[q] = xr[q] + rr[q] * it;
        if (t == deg - 1) break;
        c128* rs = lds_poly + (t & 1) * N;
#pragma unroll
        for (int q = 0; q < POLY_NPT; ++q) {
            int n = threadIdx.x + q * POLY_THREADS;
            if (n < N) rs[n] = rr[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < POLY_NPT; ++q) {
            int n = threadIdx.x + q * POLY_THREADS;
            if (n >= N) continue;
            const int i = ii[q], k = kk[q];
            const c128 zero = mk(0.0, 0.0);
            c128 w = k > 0 ? rs[n - 1] : zero, e = k + 1 < nx ? rs[n + 1] : zero;
            c128 nn = i > 0 ? rs[n - nx] : zero, sv = i + 1 < nz ? rs[n + nx] : zero;
            const bool lx = k == nx - 1, lz = i == nz - 1;
            double cw = lx ? sten.axl : sten.ax, cn = lz ? sten.azl : sten.az;
            c128 pr = sd[q] * rr[q] - cw * w - sten.ax * e - cn * nn - sten.az * sv;
            rr[q] = rr[q] - pr * it;
        }
    }
#pragma unroll
    for (int q = 0; q < POLY_NPT; ++q) {
        int n = threadIdx.x + q * POLY_THREADS;
        if (n < N) out[n] = ccast<T>(xr[q]);
    }
}

// Whole-wave DPP lane shifts (lane l receives the value of lane l - 1, resp.
// l + 1; the lane without a source receives zero), on the two 32-bit halves of
// each double.
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ c128 lane_shift(c128 v) {
    return mk(lane_shift<CTRL>(v.re), lane_shift<CTRL>(v.im));
}

// The same polynomial for levels of at most 64 x 64 nodes (the coarsest level of
// a 256 x 256 grid with three levels), laid out by rows: wave w of the
// 1024-thread workgroup holds rows PW_ROWS w .. PW_ROWS w + 3, lane k column k.
// A node's west and east neighbours then come from the adjacent lanes by DPP
// shifts and its north and south ones from the thread's own registers; only the
// strips' edge rows cross waves, through LDS (each wave writes its top and
// bottom rows, double buffered as in k_poly_lds, one barrier per factor, and
// reads the rows next to its strip).  Per thread and factor that is 2 LDS
// writes and 2 reads where k_poly_lds has 4 and 16.  The per-node arithmetic,
// its order and the boundary coefficients are those of k_poly_lds; lanes and
// rows outside the level hold zeros throughout.
constexpr int PW_ROWS = 4, PW_WAVES = POLY_THREADS / 64, PW_MAXNX = 64, PW_MAXNZ = PW_WAVES * PW_ROWS;
template <typename T>
__global__ __launch_bounds__(POLY_THREADS) void k_poly_rows(const cx<T>* __restrict__ src, cx<T>* __restrict__ out,
                                                            const c128* __restrict__ sl, int nz, int nx,
                                                            Sten<double> sten, const c128* __restrict__ roots,
                                                            int deg, const RhsState* __restrict__ st, int rhs0,
                                                            unsigned long long* wc) {
    const int rl = blockIdx.x;
    if (st) {
        const RhsState& S = st[rhs0 + rl];
        if (!S.active || S.cycdone) return;
    }
    const int N = nz * nx;
    src += (long)rl * N;
    out += (long)rl * N;
    add_work(wc, (unsigned long long)N * 2 * sizeof(cx<T>));
    __shared__ c128 inv_roots[64];                  // 1 / theta_t (deg <= 64)
    __shared__ c128 edge[2][PW_WAVES][2][64];       // [buffer][wave][top, bottom row][column]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < deg) {
        const c128 th = roots[threadIdx.x];
        const double d = th.re * th.re + th.im * th.im;
        inv_roots[threadIdx.x] = mk(th.re / d, -th.im / d);
    }
    const c128 zero = mk(0.0, 0.0);
    c128 xr[PW_ROWS], rr[PW_ROWS], sd[PW_ROWS];
    double cn[PW_ROWS];
    bool ok[PW_ROWS];
    const double cw = lane == nx - 1 ? sten.axl : sten.ax;
#pragma unroll
    for (int q = 0; q < PW_ROWS; ++q) {
        const int i = wave * PW_ROWS + q, n = i * nx + lane;
        ok[q] = lane < nx && i < nz;
        cn[q] = i == nz - 1 ? sten.azl : sten.az;
        xr[q] = zero;
        rr[q] = zero;
        sd[q] = zero;
        if (ok[q]) {
            rr[q] = ccast<double>(src[n]);
            // stencil diagonal minus the mass term
            NodeSten<double> ns = node_sten(sten, i, lane, nz, nx);
            sd[q] = mk(ns.dg - sl[n].re, -sl[n].im);
        }
    }
    __syncthreads();
    for (int t = 0; t < deg; ++t) {
        const c128 it = inv_roots[t];
#pragma unroll
        for (int q = 0; q < PW_ROWS; ++q) xr[q] = xr[q] + rr[q] * it;
        if (t == deg - 1) break;
        c128(*eb)[2][64] = edge[t & 1];
        eb[wave][0][lane] = rr[0];
        eb[wave][1][lane] = rr[PW_ROWS - 1];
        c128 wv[PW_ROWS], ev[PW_ROWS];
#pragma unroll
        for (int q = 0; q < PW_ROWS; ++q) {
            wv[q] = lane_shift<DPP_WAVE_SHR1>(rr[q]);
            ev[q] = lane_shift<DPP_WAVE_SHL1>(rr[q]);
        }
        __syncthreads();
        const c128 above = wave > 0 ? eb[wave - 1][1][lane] : zero;
        const c128 below = wave + 1 < PW_WAVES ? eb[wave + 1][0][lane] : zero;
        c128 rn[PW_ROWS];
#pragma unroll
        for (int q = 0; q < PW_ROWS; ++q) {
            const c128 nn = q > 0 ? rr[q - 1] : above;
            const c128 sv = q + 1 < PW_ROWS ? rr[q + 1] : below;
            c128 pr = sd[q] * rr[q] - cw * wv[q] - sten.ax * ev[q] - cn[q] * nn - sten.az * sv;
            rn[q] = ok[q] ? rr[q] - pr * it : zero;
        }
#pragma unroll
        for (int q = 0; q < PW_ROWS; ++q) rr[q] = rn[q];
    }
#pragma unroll
    for (int q = 0; q < PW_ROWS; ++q)
        if (ok[q]) out[(wave * PW_ROWS + q) * nx + lane] = ccast<T>(xr[q]);
}

template <typename T>
static const cx<T>* sl_of(const Level& L) {
    if constexpr (sizeof(T) == 4)
        return L.sl32;
    else
        return L.sl64;
}
template <typename T>
static const cx<T>* wd_of(const Level& L) {
    if constexpr (sizeof(T) == 4)
        return L.wd32;
    else
        return L.wd64;
}

template <typename T>
size_t mg_work_elems(const helm_op* op, int level) {
    return (size_t)op->lv[level].n();
}
template size_t mg_work_elems<float>(const helm_op*, int);
template size_t mg_work_elems<double>(const helm_op*, int);

template <typename T>
int launch_vcycle(const helm_op* op, const cx<T>* f, const double* fscale, int fstride, cx<T>* out,
                  const cx<T>* addend, int nrhs, const RhsState* st, int rhs0, MgWork<T>& w, hipStream_t s) {
    const int L = op->nlev;
    const T wj = T(op->jw);
    for (int r0 = 0; r0 < nrhs; r0 += 65535) {
        int nr = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        long off0 = (long)r0 * op->n();
        // restriction chain
        for (int l = 0; l + 1 < L; ++l) {
            const Level& F = op->lv[l];
            const Level& C = op->lv[l + 1];
            const cx<T>* fin = l == 0 ? f + off0 : w.f[l] + (long)r0 * F.n();
            dim3 grid((C.nx + MG_T - 1) / MG_T, (C.nz + MG_T - 1) / MG_T, nr);
            TIMED_LAUNCH("k_mg_down", s, k_mg_down<T>, grid, dim3(256), 0, s, fin, l == 0 ? fscale : nullptr,
                         fstride, wd_of<T>(F), F.nz, F.nx, F.sten<T>(), wj, w.f[l + 1] + (long)r0 * C.n(), C.nz,
                         C.nx, st, rhs0 + r0, WORK_COUNTER("k_mg_down", s));
            HELM_CHECK_LAUNCH();
        }
        // coarsest level: x = p(P) f
        {
            const int l = L - 1;
            const Level& C = op->lv[l];
            long n = C.n();
            const cx<T>* src = l == 0 ? f + off0 : w.f[l] + (long)r0 * n;
            cx<T>* xdst = l == 0 ? out + off0 : w.e[l] + (long)r0 * n;
            dim3 grid((unsigned)((n + 255) / 256), nr);
            const int deg = (int)op->roots.size();
            c128* bufs[2] = {w.ra + (long)r0 * n, w.rb + (long)r0 * n};
            c128* xw = w.xw + (long)r0 * n;
            if (l == 0 && (fscale || addend))
                return fail(HELM_EINVAL, "single-level cycle does not take scaled or offset inputs");
            if (C.nx <= PW_MAXNX && C.nz <= PW_MAXNZ && op->roots_dev) {
                TIMED_LAUNCH("k_poly_rows", s, k_poly_rows<T>, dim3(nr), dim3(POLY_THREADS), 0, s, src, xdst, C.sl64,
                             C.nz, C.nx, C.sten<double>(), op->roots_dev, deg, st, rhs0 + r0,
                             WORK_COUNTER("k_poly_rows", s));
                HELM_CHECK_LAUNCH();
            } else if (n <= POLY_LDS_MAX && op->roots_dev && op->poly_lds_ok) {
                size_t lds = 2 * (size_t)n * sizeof(c128);
                TIMED_LAUNCH("k_poly_lds", s, k_poly_lds<T>, dim3(nr), dim3(POLY_THREADS), lds, s, src, xdst, C.sl64,
                             C.nz, C.nx, C.sten<double>(), op->roots_dev, deg, st, rhs0 + r0,
                             WORK_COUNTER("k_poly_lds", s));
                HELM_CHECK_LAUNCH();
            } else
            for (int t = 0; t < deg; ++t) {
                c128 th = op->roots[t];
                double d = th.re * th.re + th.im * th.im;
                c128 it = mk(th.re / d, -th.im / d);
                const c128* rin = bufs[(t + 1) & 1];
                c128* rout = bufs[t & 1];
                TIMED_LAUNCH("k_poly_term", s, k_poly_term<T>, grid, dim3(256), 0, s, src, rin, rout, xw, xdst,
                             C.sl64, C.nz, C.nx, C.sten<double>(), it, t == 0 ? 1 : 0, t == deg - 1 ? 1 : 0, st,
                             rhs0 + r0, WORK_COUNTER("k_poly_term", s));
                HELM_CHECK_LAUNCH();
            }
        }
        // prolongation chain
        for (int l = L - 2; l >= 0; --l) {
            const Level& F = op->lv[l];
            const Level& C = op->lv[l + 1];
            const cx<T>* fin = l == 0 ? f + off0 : w.f[l] + (long)r0 * F.n();
            cx<T>* dst = l == 0 ? out + off0 : w.e[l] + (long)r0 * F.n();
            dim3 grid((F.nx + MG_T - 1) / MG_T, (F.nz + MG_T - 1) / MG_T, nr);
            TIMED_LAUNCH("k_mg_up", s, k_mg_up<T>, grid, dim3(256), 0, s, fin, l == 0 ? fscale : nullptr, fstride,
                         sl_of<T>(F), wd_of<T>(F), F.nz, F.nx, F.sten<T>(), wj, w.e[l + 1] + (long)r0 * C.n(), C.nz, C.nx, dst,
                         (l == 0 && addend) ? addend + off0 : nullptr, st, rhs0 + r0, WORK_COUNTER("k_mg_up", s));
            HELM_CHECK_LAUNCH();
        }
    }
    return HELM_OK;
}
template int launch_vcycle<float>(const helm_op*, const c64*, const double*, int, c64*, const c64*, int,
                                  const RhsState*, int, MgWork<float>&, hipStream_t);
template int launch_vcycle<double>(const helm_op*, const c128*, const double*, int, c128*, const c128*, int,
                                   const RhsState*, int, MgWork<double>&, hipStream_t);

// ------------------------------------------------------------------ FGMRES kernels
template <typename T>
void fill_group(GroupArgs<T>& g, const helm_op* op, int rhs0, long off0) {
    g.nz = op->nz;
    g.nx = op->nx;
    g.N = op->n();
    g.nblk = (int)((g.N / 2 + PAIRS_PER_BLOCK - 1) / PAIRS_PER_BLOCK);
    g.rhs0 = rhs0;
    g.off0 = off0;
    g.ax = T(1.0 / (op->hx * op->hx));
    g.az = T(1.0 / (op->hz * op->hz));
    if constexpr (sizeof(T) == 4)
        g.coef = op->coef32;
    else
        g.coef = op->coef64;
    g.k2 = op->lv[0].k2;
    g.gam = op->lv[0].g;
    g.omega2 = op->omega * op->omega;
    g.axd = 1.0 / (op->hx * op->hx);
    g.azd = 1.0 / (op->hz * op->hz);
}
template void fill_group<float>(GroupArgs<float>&, const helm_op*, int, long);
template void fill_group<double>(GroupArgs<double>&, const helm_op*, int, long);

// Block-wide sum of K complex values per thread (acc[k]) into part[k] (thread 0..K-1 write).
template <int NW>
__device__ __forceinline__ void block_sum_store(double (*lds)[NW][2], int k, double re, double im) {
    re = wave_sum(re);
    im = wave_sum(im);
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
    if (ln == 0) {
        lds[k][wv][0] = re;
        lds[k][wv][1] = im;
    }
}

constexpr int NWV = VEC_THREADS / WAVE;  // waves per block

// res[k] = sum over blocks b of part[b*K + k], k < nk, deterministic: thread
// (slot, k) sums blocks b = slot, slot + nslot, ... in order (all loads of a
// thread are independent, so they are in flight together), then thread k
// sums the slots in order.  The result lands in LDS.
__device__ __forceinline__ void fold_partials(const c128* __restrict__ part, int nblk, int K, int nk, c128* res) {
    __shared__ c128 slots[VEC_THREADS];
    const int nslot = VEC_THREADS / nk;
    const int slot = threadIdx.x / nk, k = threadIdx.x - slot * nk;
    if (slot < nslot) {
        double re = 0, im = 0;
        for (int b = slot; b < nblk; b += nslot) {
            c128 v = part[(long)b * K + k];
            re += v.re;
            im += v.im;
        }
        slots[threadIdx.x] = mk(re, im);
    }
    __syncthreads();
    if (threadIdx.x < nk) {
        c128 s = mk(0.0, 0.0);
        for (int sl = 0; sl < nslot; ++sl) s = s + slots[sl * nk + threadIdx.x];
        res[threadIdx.x] = s;
    }
    __syncthreads();
}

// Nodes of one RHS covered by this level-0 block.
__device__ __forceinline__ unsigned long long block_nodes(long N) {
    long q0 = (long)blockIdx.x * PAIRS_PER_BLOCK;
    long np = N / 2 - q0;
    return 2ull * (unsigned long long)(np < PAIRS_PER_BLOCK ? np : PAIRS_PER_BLOCK);
}

// Block partials of the vector kernels go to part[r][blk][0..K) (K = m+2);
// k_reduce (one workgroup per RHS) folds them in a fixed order and takes the
// scalar decisions.  No kernel synchronises across its own blocks: the kernel
// boundary is what makes the partials visible.
__device__ __forceinline__ void store_partials(double (*lds)[NWV][2], int nk, c128* __restrict__ part) {
    __syncthreads();
    if (threadIdx.x < nk) {
        c128 p = mk(0.0, 0.0);
        for (int w = 0; w < NWV; ++w) p = p + mk(lds[threadIdx.x][w][0], lds[threadIdx.x][w][1]);
        part[threadIdx.x] = p;
    }
}

// r = b - H x in FP64; V0 = r; partials (||r||^2, ||b||^2).
template <typename T>
__global__ __launch_bounds__(256) void k_true_residual(GroupArgs<T> g, SolveArgs<T> a, unsigned long long* wc) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (S.done) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    double rr = 0, bb = 0;
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= g.N / 2) continue;
        long n0 = 2 * q;
        int i = (int)(n0 / g.nx), k0 = (int)(n0 - (long)i * g.nx);
        double m0 = g.k2[n0], m1 = g.k2[n0 + 1];
        double g0 = g.gam[n0], g1 = g.gam[n0 + 1];
        c128 c0 = mk(g.omega2 * m0, -g.omega2 * m0 * g0);
        c128 c1 = mk(g.omega2 * m1, -g.omega2 * m1 * g1);
        if (a.conjop) {
            c0 = conj(c0);
            c1 = conj(c1);
        }
        pair2<double> hx = stencil_pair<double, double>(a.x + base, n0, i, k0, g.nz, g.nx, g.axd, g.azd, c0, c1);
        pair2<float> bv = ld_pair(a.b + base + n0);
        c128 r0 = ccast<double>(bv.a) - hx.a, r1 = ccast<double>(bv.b) - hx.b;
        rr += norm2(r0) + norm2(r1);
        bb += norm2(bv.a) + norm2(bv.b);
        pair2<T> out = {ccast<T>(r0), ccast<T>(r1)};
        st_pair(a.V + base + n0, out);
    }
    add_work(wc, block_nodes(g.N) * (24 + 2 * sizeof(T)));
    __shared__ double lds[1][NWV][2];
    block_sum_store<NWV>(lds, 0, rr, bb);
    store_partials(lds, 1, a.part + ((long)r * a.maxblk + blockIdx.x) * (a.m + 2));
}

// w = H z_j -> V[j+1]; partials <v_i, w> (i <= j) and ||w||^2.
template <typename T>
__global__ __launch_bounds__(256) void k_matvec_dot(GroupArgs<T> g, SolveArgs<T> a, int j, unsigned long long* wc) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active || S.cycdone) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    const cx<T>* z = a.Z + (long)j * a.Ntot + base;
    cx<T>* w = a.V + (long)(j + 1) * a.Ntot + base;
    pair2<T> wv[2];
    bool ok[2];
    T ww = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        ok[h] = q < g.N / 2;
        wv[h] = {mk(T(0), T(0)), mk(T(0), T(0))};
        if (!ok[h]) continue;
        long n0 = 2 * q;
        int i = (int)(n0 / g.nx), k0 = (int)(n0 - (long)i * g.nx);
        pair2<T> c = ld_pair(g.coef + n0);
        if (a.conjop) {
            c.a = conj(c.a);
            c.b = conj(c.b);
        }
        wv[h] = stencil_pair<T, T>(z, n0, i, k0, g.nz, g.nx, g.ax, g.az, c.a, c.b);
        st_pair(w + n0, wv[h]);
        ww += norm2(wv[h].a) + norm2(wv[h].b);
    }
    add_work(wc, block_nodes(g.N) * (j + 3) * 2 * sizeof(T));
    __shared__ double lds[MAX_RESTART + 2][NWV][2];
    for (int i = 0; i <= j; ++i) {
        const cx<T>* vi = a.V + (long)i * a.Ntot + base;
        cx<T> acc = mk(T(0), T(0));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!ok[h]) continue;
            long n0 = 2 * ((long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x);
            pair2<T> v = ld_pair(vi + n0);
            acc = acc + cdot1(v.a, wv[h].a) + cdot1(v.b, wv[h].b);
        }
        block_sum_store<NWV>(lds, i, (double)acc.re, (double)acc.im);
    }
    block_sum_store<NWV>(lds, j + 1, (double)ww, 0.0);
    store_partials(lds, j + 2, a.part + ((long)r * a.maxblk + blockIdx.x) * (a.m + 2));
}

// Second Gram-Schmidt pass: partials <v_i, w>, only where requested.
template <typename T>
__global__ __launch_bounds__(256) void k_dot2(GroupArgs<T> g, SolveArgs<T> a, int j, unsigned long long* wc) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active || S.cycdone || !S.need2) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    const cx<T>* w = a.V + (long)(j + 1) * a.Ntot + base;
    pair2<T> wv[2];
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        ok[h] = q < g.N / 2;
        wv[h] = ok[h] ? ld_pair(w + 2 * q) : pair2<T>{mk(T(0), T(0)), mk(T(0), T(0))};
    }
    add_work(wc, block_nodes(g.N) * (j + 2) * 2 * sizeof(T));
    __shared__ double lds[MAX_RESTART + 2][NWV][2];
    for (int i = 0; i <= j; ++i) {
        const cx<T>* vi = a.V + (long)i * a.Ntot + base;
        cx<T> acc = mk(T(0), T(0));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!ok[h]) continue;
            long n0 = 2 * ((long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x);
            pair2<T> v = ld_pair(vi + n0);
            acc = acc + cdot1(v.a, wv[h].a) + cdot1(v.b, wv[h].b);
        }
        block_sum_store<NWV>(lds, i, (double)acc.re, (double)acc.im);
    }
    store_partials(lds, j + 1, a.part + ((long)r * a.maxblk + blockIdx.x) * (a.m + 2));
}

// Givens update of column j of the Hessenberg matrix (FP64), one thread.
template <typename T>
__device__ void givens_finalize(const SolveArgs<T>& a, RhsState& S, int r, int j, double hn) {
    const int m = a.m;
    c128* col = a.H + ((long)r * m + j) * (m + 1);
    c128* cs = a.cs + (long)r * m;
    c128* sn = a.sn + (long)r * m;
    c128* gg = a.g + (long)r * (m + 1);
    col[j + 1] = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        c128 t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = conj(cs[i]) * col[i + 1] - conj(sn[i]) * col[i];
        col[i] = t;
    }
    c128 av = col[j], cv = col[j + 1];
    double den = sqrt(norm2(av) + norm2(cv));
    c128 c, s;
    if (den == 0.0) {
        c = mk(1.0, 0.0);
        s = mk(0.0, 0.0);
    } else {
        c = (1.0 / den) * conj(av);
        s = (1.0 / den) * conj(cv);
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = c * av + s * cv;
    col[j + 1] = mk(0.0, 0.0);
    c128 gj = gg[j];
    gg[j + 1] = mk(0.0, 0.0) - conj(s) * gj;
    gg[j] = c * gj;
    S.jlen = j + 1;
    S.iters += 1;
    double est = sqrt(norm2(gg[j + 1])) / S.bnorm;
    S.est = est;
    a.vscale[(long)r * (m + 1) + j + 1] = hn > 0 ? 1.0 / hn : 0.0;
    if (!(hn > 0.0) || !(est > a.tol) || S.iters >= S.maxit) S.cycdone = 1;
}

// w -= sum_i hcur_i v_i (in place in V[j+1]); partial ||w||^2.
template <typename T>
__global__ __launch_bounds__(256) void k_update(GroupArgs<T> g, SolveArgs<T> a, int j, int pass, unsigned long long* wc) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active || S.cycdone) return;
    if (pass == 2 && !S.need2) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    cx<T>* w = a.V + (long)(j + 1) * a.Ntot + base;
    __shared__ cx<T> hc[MAX_RESTART + 1];
    if (threadIdx.x <= j) {
        c128 hv = a.hcur[(long)r * (a.m + 1) + threadIdx.x];
        double sc = a.vscale[(long)r * (a.m + 1) + threadIdx.x];
        hc[threadIdx.x] = mk(T(hv.re * sc), T(hv.im * sc));
    }
    __syncthreads();
    T ww = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= g.N / 2) continue;
        long n0 = 2 * q;
        pair2<T> wv = ld_pair(w + n0);
        for (int i = 0; i <= j; ++i) {
            pair2<T> v = ld_pair(a.V + (long)i * a.Ntot + base + n0);
            wv.a = wv.a - hc[i] * v.a;
            wv.b = wv.b - hc[i] * v.b;
        }
        st_pair(w + n0, wv);
        ww += norm2(wv.a) + norm2(wv.b);
    }
    add_work(wc, block_nodes(g.N) * (j + 3) * 2 * sizeof(T));
    __shared__ double lds[1][NWV][2];
    block_sum_store<NWV>(lds, 0, (double)ww, 0.0);
    store_partials(lds, 1, a.part + ((long)r * a.maxblk + blockIdx.x) * (a.m + 2));
}

// Per-RHS fold of the block partials (one workgroup per RHS) and the scalar
// steps that follow each vector kernel:
//   RED_RESID  (after k_true_residual): cycle start, convergence decision;
//   RED_DOTS   (after k_matvec_dot):    hcur = first-pass coefficients, wb2;
//   RED_DOTS2  (after k_dot2):          hcur = second-pass coefficients;
//   RED_NORM1/2 (after k_update pass 1/2): Hessenberg column, reorthogonalisation
//               decision, Givens rotation.
enum { RED_RESID = 0, RED_DOTS = 1, RED_DOTS2 = 2, RED_NORM1 = 3, RED_NORM2 = 4 };

template <typename T>
__global__ __launch_bounds__(256) void k_reduce(SolveArgs<T> a, int rhs0, int nblk, int mode, int j) {
    const int r = rhs0 + blockIdx.x;
    RhsState& S = a.st[r];
    if (mode == RED_RESID) {
        if (S.done) return;
    } else {
        if (!S.active || S.cycdone) return;
        if ((mode == RED_DOTS2 || mode == RED_NORM2) && !S.need2) return;
    }
    const int K = a.m + 2;
    const int nk = mode == RED_DOTS ? j + 2 : mode == RED_DOTS2 ? j + 1 : 1;
    __shared__ c128 red[MAX_RESTART + 2];
    fold_partials(a.part + (long)r * a.maxblk * K, nblk, K, nk, red);
    const long ro = (long)r * (a.m + 1);
    if (mode == RED_DOTS || mode == RED_DOTS2) {
        if (threadIdx.x <= j) a.hcur[ro + threadIdx.x] = a.vscale[ro + threadIdx.x] * red[threadIdx.x];
        if (mode == RED_DOTS && threadIdx.x == j + 1) S.wb2 = red[j + 1].re;
        return;
    }
    if (threadIdx.x != 0) return;
    if (mode == RED_RESID) {
        c128 s = red[0];
        double beta = sqrt(s.re);
        if (S.cycles == 0) S.bnorm = sqrt(s.im);
        S.cycles += 1;
        S.active = 0;
        S.cycdone = 0;
        S.jlen = 0;
        S.need2 = 0;
        if (S.bnorm == 0.0) {
            S.relres = 0.0;
            S.status = HELM_OK;
            S.done = 1;
        } else {
            S.relres = beta / S.bnorm;
            if (!(beta == beta) || isinf(beta)) {
                S.status = HELM_ENAN;
                S.done = 1;
            } else if (S.relres <= a.tol) {
                S.status = HELM_OK;
                S.done = 1;
            } else if (S.iters >= S.maxit) {
                S.status = HELM_NOT_CONVERGED;
                S.done = 1;
            } else {
                S.active = 1;
                a.g[ro] = mk(beta, 0.0);
                a.vscale[ro] = 1.0 / beta;
            }
        }
        return;
    }
    // RED_NORM1 / RED_NORM2
    const int pass = mode == RED_NORM1 ? 1 : 2;
    double s2 = red[0].re;
    c128* col = a.H + ((long)r * a.m + j) * (a.m + 1);
    for (int i = 0; i <= j; ++i) {
        c128 hv = a.hcur[ro + i];
        col[i] = pass == 1 ? hv : col[i] + hv;
    }
    if (pass == 1 && a.reorth && s2 < 0.49 * S.wb2) {
        S.need2 = 1;
    } else {
        S.need2 = 0;
        givens_finalize(a, S, r, j, sqrt(s2));
    }
}

// y = R^-1 g for each active RHS (back substitution, FP64): one block per RHS
// stages the triangle in LDS with parallel loads, then one lane substitutes.
template <typename T>
__global__ __launch_bounds__(256) void k_lsq(SolveArgs<T> a) {
    const int r = blockIdx.x;
    const RhsState& S = a.st[r];
    if (!S.active) return;
    const int m = a.m, k = S.jlen;
    __shared__ c128 R[MAX_RESTART * (MAX_RESTART + 1)];
    __shared__ c128 gl[MAX_RESTART + 1];
    const c128* Hr = a.H + (long)r * m * (m + 1);
    for (int t = threadIdx.x; t < k * (m + 1); t += blockDim.x) R[t] = Hr[t];
    for (int t = threadIdx.x; t < k; t += blockDim.x) gl[t] = a.g[(long)r * (m + 1) + t];
    __syncthreads();
    if (threadIdx.x != 0) return;
    c128* y = a.y + (long)r * m;
    __shared__ c128 yl[MAX_RESTART];
    for (int i = k - 1; i >= 0; --i) {
        c128 s = gl[i];
        for (int l = i + 1; l < k; ++l) s = s - R[l * (m + 1) + i] * yl[l];
        yl[i] = s * cinv(R[i * (m + 1) + i]);
    }
    for (int i = 0; i < k; ++i) y[i] = yl[i];
}

// x += sum_i y_i z_i (x in c128).
template <typename T>
__global__ __launch_bounds__(256) void k_sol_update(GroupArgs<T> g, SolveArgs<T> a, unsigned long long* wc) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    const int k = S.jlen;
    __shared__ c128 ys[MAX_RESTART];
    if (threadIdx.x < k) ys[threadIdx.x] = a.y[(long)r * a.m + threadIdx.x];
    __syncthreads();
    add_work(wc, block_nodes(g.N) * (32 + k * 2 * sizeof(T)));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= g.N / 2) continue;
        long n0 = 2 * q;
        pair2<double> xv = ld_pair(a.x + base + n0);
        for (int i = 0; i < k; ++i) {
            pair2<T> zv = ld_pair(a.Z + (long)i * a.Ntot + base + n0);
            xv.a = xv.a + ys[i] * ccast<double>(zv.a);
            xv.b = xv.b + ys[i] * ccast<double>(zv.b);
        }
        st_pair(a.x + base + n0, xv);
    }
}

// z_j = vscale_j v_j (identity preconditioner).
template <typename T>
__global__ __launch_bounds__(256) void k_scale_copy(GroupArgs<T> g, SolveArgs<T> a, int j) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active || S.cycdone) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    const T sc = T(a.vscale[(long)r * (a.m + 1) + j]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= g.N / 2) continue;
        long n0 = 2 * q;
        pair2<T> v = ld_pair(a.V + (long)j * a.Ntot + base + n0);
        v.a = sc * v.a;
        v.b = sc * v.b;
        st_pair(a.Z + (long)j * a.Ntot + base + n0, v);
    }
}

// out = vscale_j v_j - H e0  (fine-level residual of the network's guess)
template <typename T>
__global__ __launch_bounds__(256) void k_residual_vs_e0(GroupArgs<T> g, SolveArgs<T> a, int j,
                                                        const cx<T>* __restrict__ e0, cx<T>* __restrict__ out) {
    const int r = g.rhs0 + blockIdx.y;
    const RhsState& S = a.st[r];
    if (!S.active || S.cycdone) return;
    const long base = g.off0 + (long)blockIdx.y * g.N;
    const long lbase = (long)blockIdx.y * g.N;
    const T sc = T(a.vscale[(long)r * (a.m + 1) + j]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        long q = (long)blockIdx.x * PAIRS_PER_BLOCK + h * VEC_THREADS + threadIdx.x;
        if (q >= g.N / 2) continue;
        long n0 = 2 * q;
        int i = (int)(n0 / g.nx), k0 = (int)(n0 - (long)i * g.nx);
        pair2<T> c = ld_pair(g.coef + n0);
        if (a.conjop) {
            c.a = conj(c.a);
            c.b = conj(c.b);
        }
        pair2<T> he = stencil_pair<T, T>(e0 + lbase, n0, i, k0, g.nz, g.nx, g.ax, g.az, c.a, c.b);
        pair2<T> v = ld_pair(a.V + (long)j * a.Ntot + base + n0);
        pair2<T> o = {sc * v.a - he.a, sc * v.b - he.b};
        st_pair(out + lbase + n0, o);
    }
}

__global__ void k_init_state(RhsState* st, int nrhs, const int* maxit_rhs, int maxit) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrhs) st[r].maxit = maxit_rhs ? maxit_rhs[r] : maxit;
}

int launch_init_state(RhsState* st, int nrhs, const int* maxit_rhs, int maxit, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3((nrhs + 255) / 256), dim3(256), 0, s, st, nrhs, maxit_rhs, maxit);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

__global__ void k_zero_done_x(int nblk, long N, long off0, int rhs0, const RhsState* st, c128* x) {
    const int r = rhs0 + blockIdx.y;
    if (!(st[r].done && st[r].bnorm == 0.0)) return;
    long n = (long)blockIdx.x * 256 + threadIdx.x;
    if (n < N) x[off0 + (long)blockIdx.y * N + n] = mk(0.0, 0.0);
    (void)nblk;
}

// ------------------------------------------------------------------ launchers
template <typename T>
static int launch_reduce(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int mode, int j, hipStream_t s) {
    TIMED_LAUNCH("k_reduce", s, k_reduce<T>, dim3(ng), dim3(VEC_THREADS), 0, s, a, g.rhs0, g.nblk, mode, j);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

template <typename T>
int launch_true_residual(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, hipStream_t s) {
    TIMED_LAUNCH("k_true_residual", s, k_true_residual<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a,
                 WORK_COUNTER("k_true_residual", s));
    HELM_CHECK_LAUNCH();
    return launch_reduce<T>(g, ng, a, RED_RESID, 0, s);
}
template <typename T>
int launch_matvec_dot(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s) {
    TIMED_LAUNCH("k_matvec_dot", s, k_matvec_dot<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a, j,
                 WORK_COUNTER("k_matvec_dot", s));
    HELM_CHECK_LAUNCH();
    return launch_reduce<T>(g, ng, a, RED_DOTS, j, s);
}
template <typename T>
int launch_update(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, int pass, hipStream_t s) {
    TIMED_LAUNCH("k_update", s, k_update<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a, j, pass,
                 WORK_COUNTER("k_update", s));
    HELM_CHECK_LAUNCH();
    return launch_reduce<T>(g, ng, a, pass == 1 ? RED_NORM1 : RED_NORM2, j, s);
}
template <typename T>
int launch_dot2(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s) {
    TIMED_LAUNCH("k_dot2", s, k_dot2<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a, j,
                 WORK_COUNTER("k_dot2", s));
    HELM_CHECK_LAUNCH();
    return launch_reduce<T>(g, ng, a, RED_DOTS2, j, s);
}
template <typename T>
int launch_lsq(const SolveArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_lsq<T>, dim3(a.nrhs), dim3(256), 0, s, a);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}
template <typename T>
int launch_sol_update(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, hipStream_t s) {
    TIMED_LAUNCH("k_sol_update", s, k_sol_update<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a,
                 WORK_COUNTER("k_sol_update", s));
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}
template <typename T>
int launch_scale_copy(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a, j);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}
template <typename T>
int launch_residual_vs_e0(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, const cx<T>* e0,
                          cx<T>* out, hipStream_t s) {
    hipLaunchKernelGGL(k_residual_vs_e0<T>, dim3(g.nblk, ng), dim3(VEC_THREADS), 0, s, g, a, j, e0, out);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}
int launch_zero_done_x(const GroupArgs<double>& g, int ng, const RhsState* st, c128* x, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_done_x, dim3((unsigned)((g.N + 255) / 256), ng), dim3(256), 0, s, g.nblk, g.N,
                       g.off0, g.rhs0, st, x);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

#define INST(T)                                                                                              \
    template int launch_true_residual<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, hipStream_t);        \
    template int launch_matvec_dot<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, int, hipStream_t);      \
    template int launch_update<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, int, int, hipStream_t);     \
    template int launch_dot2<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, int, hipStream_t);            \
    template int launch_lsq<T>(const SolveArgs<T>&, hipStream_t);                                            \
    template int launch_sol_update<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, hipStream_t);           \
    template int launch_scale_copy<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, int, hipStream_t);      \
    template int launch_residual_vs_e0<T>(const GroupArgs<T>&, int, const SolveArgs<T>&, int, const cx<T>*, \
                                          cx<T>*, hipStream_t);
INST(float)
INST(double)

}  // namespace helm
