// Host-side small dense linear algebra for the coarsest-level polynomial:
// Arnoldi on the coarsest shifted Laplacian, harmonic Ritz values, complex
// Hessenberg QR eigenvalues, Leja ordering.  All FP64.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"
#include "philox.h"

namespace helm {

using zc = std::complex<double>;

// Eigenvalues of an n x n complex upper-Hessenberg matrix A (row-major) by
// the shifted QR algorithm with Wilkinson shifts and deflation.
std::vector<c128> hessenberg_eigvals(std::vector<c128> Ain, int n) {
    std::vector<zc> A(n * n);
    for (int i = 0; i < n * n; ++i) A[i] = zc(Ain[i].re, Ain[i].im);
    auto at = [&](int i, int j) -> zc& { return A[i * n + j]; };
    std::vector<zc> ev(n);
    int hi = n - 1, iter = 0;
    const double eps = 1e-15;
    std::vector<zc> rc(n), rs(n);
    while (hi >= 0) {
        if (hi == 0) {
            ev[0] = at(0, 0);
            break;
        }
        int l = hi;
        while (l > 0) {
            double sc = std::abs(at(l - 1, l - 1)) + std::abs(at(l, l));
            if (std::abs(at(l, l - 1)) <= eps * (sc > 0 ? sc : 1.0)) break;
            --l;
        }
        if (l == hi) {
            ev[hi] = at(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        ++iter;
        zc a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        zc tr = a + d, det = a * d - b * c;
        zc disc = std::sqrt(tr * tr / 4.0 - det);
        zc m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
        zc mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        if (iter % 11 == 10) mu = d + std::abs(c) * 0.75;  // exceptional shift
        if (iter > 10000) break;
        for (int k = l; k <= hi; ++k) at(k, k) -= mu;
        // QR by Givens: rotations G_k act on rows k, k+1
        for (int k = l; k < hi; ++k) {
            zc x = at(k, k), y = at(k + 1, k);
            double den = std::sqrt(std::norm(x) + std::norm(y));
            zc cc = den == 0 ? zc(1, 0) : std::conj(x) / den;
            zc ss = den == 0 ? zc(0, 0) : std::conj(y) / den;
            rc[k] = cc;
            rs[k] = ss;
            for (int j = k; j < n; ++j) {
                zc u = at(k, j), v = at(k + 1, j);
                at(k, j) = cc * u + ss * v;
                at(k + 1, j) = -std::conj(ss) * u + std::conj(cc) * v;
            }
        }
        // R Q: apply G_k^H on columns k, k+1
        for (int k = l; k < hi; ++k) {
            zc cc = rc[k], ss = rs[k];
            for (int i = 0; i <= std::min(k + 1, hi); ++i) {
                zc u = at(i, k), v = at(i, k + 1);
                at(i, k) = u * std::conj(cc) + v * std::conj(ss);
                at(i, k + 1) = -u * ss + v * cc;
            }
        }
        for (int k = l; k <= hi; ++k) at(k, k) += mu;
    }
    std::vector<c128> out(n);
    for (int i = 0; i < n; ++i) out[i] = mk(ev[i].real(), ev[i].imag());
    return out;
}

std::vector<c128> leja_order(const std::vector<c128>& th) {
    const int k = (int)th.size();
    std::vector<zc> t(k);
    for (int i = 0; i < k; ++i) t[i] = zc(th[i].re, th[i].im);
    std::vector<int> order, rest;
    int first = 0;
    for (int i = 1; i < k; ++i)
        if (std::abs(t[i]) > std::abs(t[first])) first = i;
    order.push_back(first);
    for (int i = 0; i < k; ++i)
        if (i != first) rest.push_back(i);
    while (!rest.empty()) {
        int best = -1;
        double bestv = -1;
        for (int i : rest) {
            double p = 1;
            for (int o : order) p *= std::abs(t[i] - t[o]);
            if (p > bestv) {
                bestv = p;
                best = i;
            }
        }
        order.push_back(best);
        rest.erase(std::find(rest.begin(), rest.end(), best));
    }
    std::vector<c128> out(k);
    for (int i = 0; i < k; ++i) out[i] = th[order[i]];
    return out;
}

// Arnoldi (modified Gram-Schmidt) on the level's shifted Laplacian from the
// fixed Philox start vector; harmonic Ritz values; Leja order.
std::vector<c128> coarse_roots_host(const Level& L, int degree) {
    const int nz = L.nz, nx = L.nx;
    const long n = L.n();
    // a Krylov space of the level has at most n dimensions
    if (degree > n) degree = (int)n;
    std::vector<c128> slh(n);
    if (hipMemcpy(slh.data(), L.sl64, n * sizeof(c128), hipMemcpyDeviceToHost) != hipSuccess) return {};
    const Sten<double> st = L.sten<double>();
    auto apply = [&](const std::vector<zc>& u, std::vector<zc>& v) {
        for (int i = 0; i < nz; ++i)
            for (int k = 0; k < nx; ++k) {
                long p = (long)i * nx + k;
                const bool lx = k == nx - 1, lz = i == nz - 1;
                double dg = (lx ? st.dxl : 2 * st.ax) + (lz ? st.dzl : 2 * st.az);
                zc s = (dg - zc(slh[p].re, slh[p].im)) * u[p];
                if (k > 0) s -= (lx ? st.axl : st.ax) * u[p - 1];
                if (k + 1 < nx) s -= st.ax * u[p + 1];
                if (i > 0) s -= (lz ? st.azl : st.az) * u[p - nx];
                if (i + 1 < nz) s -= st.az * u[p + nx];
                v[p] = s;
            }
    };
    std::vector<std::vector<zc>> V(degree + 1, std::vector<zc>(n));
    std::vector<zc> Hh((degree + 1) * degree, 0.0);  // row-major (degree+1) x degree
    double nrm = 0;
    for (long p = 0; p < n; ++p) {
        u32x4 w = philox_at((uint64_t)p, 0, COARSE_KEY0, COARSE_KEY1);
        V[0][p] = zc(2 * philox_u01(w.v[0]) - 1, 2 * philox_u01(w.v[1]) - 1);
        nrm += std::norm(V[0][p]);
    }
    nrm = std::sqrt(nrm);
    for (auto& z : V[0]) z /= nrm;
    int k = degree;
    std::vector<zc> w(n);
    for (int j = 0; j < degree; ++j) {
        apply(V[j], w);
        double wn0 = 0;
        for (long p = 0; p < n; ++p) wn0 += std::norm(w[p]);
        wn0 = std::sqrt(wn0);
        for (int i = 0; i <= j; ++i) {
            zc h = 0;
            for (long p = 0; p < n; ++p) h += std::conj(V[i][p]) * w[p];
            Hh[i * degree + j] = h;
            for (long p = 0; p < n; ++p) w[p] -= h * V[i][p];
        }
        double hn = 0;
        for (long p = 0; p < n; ++p) hn += std::norm(w[p]);
        hn = std::sqrt(hn);
        Hh[(j + 1) * degree + j] = hn;
        if (hn <= 1e-12 * wn0) {   // L V_j lies in the span: the space is invariant
            k = j + 1;
            break;
        }
        for (long p = 0; p < n; ++p) V[j + 1][p] = w[p] / hn;
    }
    // T = H_k + |h_{k+1,k}|^2 f e_k^T with H_k^H f = e_k  (f solves a lower-triangular-ish
    // system: H_k^H is lower Hessenberg; use Gaussian elimination with partial pivoting)
    std::vector<zc> M(k * k), rhs(k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) M[i * k + j] = std::conj(Hh[j * degree + i]);
    rhs[k - 1] = 1.0;
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int r = c + 1; r < k; ++r)
            if (std::abs(M[r * k + c]) > std::abs(M[piv * k + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < k; ++j) std::swap(M[c * k + j], M[piv * k + j]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int r = c + 1; r < k; ++r) {
            zc f = M[r * k + c] / M[c * k + c];
            if (f == zc(0)) continue;
            for (int j = c; j < k; ++j) M[r * k + j] -= f * M[c * k + j];
            rhs[r] -= f * rhs[c];
        }
    }
    std::vector<zc> f(k);
    for (int r = k - 1; r >= 0; --r) {
        zc s = rhs[r];
        for (int j = r + 1; j < k; ++j) s -= M[r * k + j] * f[j];
        f[r] = s / M[r * k + r];
    }
    double hk = std::abs(Hh[k * degree + (k - 1)]);
    std::vector<c128> T(k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            zc v = Hh[i * degree + j];
            if (j == k - 1) v += hk * hk * f[i];
            T[i * k + j] = mk(v.real(), v.imag());
        }
    return leja_order(hessenberg_eigvals(T, k));
}

}  // namespace helm
