// Encoder-solver network: parameters, forward and backward programs, the
// preconditioner used inside FGMRES, training-data generation, Adam, the
// light-weight retraining, and their C entry points.
//
// Layer list (same order as the reference description of the architecture):
//   encoder: conv(2->32); 2 x resblock(32); for l = 1..3: conv_s2(w[l-1]->w[l]),
//            2 x resblock(w[l]); for l = 2..0: up(w[l+1]->w[l]), conv(2w[l]->w[l])
//            on [up, skip_l], resblock(w[l])  ->  z_0..z_3
//   solver:  conv(2->32); for l = 0..3: [l>0: conv_s2(w[l-1]->w[l])],
//            conv(2w[l]->w[l]) on [h, z_l], resblock(w[l]); for l = 2..0:
//            up(w[l+1]->w[l]), conv(2w[l]->w[l]) on [up, skip_l], resblock(w[l]);
//            conv(32->2) without activation.
// resblock(x) = x + conv2(ReLU(conv1(x))); all other convolutions are
// followed by ReLU.  Weights: conv [Cout][3][3][Cin], up [2][2][Cout][Cin],
// flat order layer by layer, W then bias.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "cnn.h"
#include "conv.h"
#include "philox.h"

namespace helm {

enum { L_CONV = 0, L_UP = 1 };

struct LayerDesc {
    int kind, cin, cout, stride;
    long woff, boff;  // offsets of W and b in the flat parameter vector
    long nw;
    int K;            // forward GEMM depth (padded to 32)
    long wb_off;      // offset of the forward bf16 weights [N][K]
    long wt_off;      // offset of the data-gradient bf16 weights [Cin][Kt]
    int Kt;           // data-gradient GEMM depth
    // solver context convolutions conv(concat(h, z)): the weights split into
    // the h part [N][Kh] and the z part [N][Kz] (inference evaluates the z part
    // once per encoder pass)
    int ctx = 0, ch = 0, Kh = 0, Kz = 0;
    long wh_off = 0, wz_off = 0;
};

static int pad32(int k) { return (k + 31) / 32 * 32; }

}  // namespace helm

using namespace helm;

struct cnn_net {
    int widths[4] = {32, 64, 128, 256};
    int down_res = 2;
    std::vector<LayerDesc> layers;
    int n_enc = 0;
    long nparam = 0;
    long nwb = 0;
    float* master = nullptr;   // fp32 parameters
    float* grad = nullptr;     // fp32 gradients
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    long adam_t = 0;
    bf16* wb = nullptr;        // bf16 forward and data-gradient weight copies
    uint64_t version = 1;      // bumped whenever the parameters change
    uint64_t uid = 0;          // process-unique id (encoder contexts are keyed by it)
    uint64_t seed = 0;
};

namespace helm {

// ------------------------------------------------------------------ layer table
static void build_layers(cnn_net* n) {
    const int* w = n->widths;
    auto add = [&](int kind, int cin, int cout, int stride, int ctx = 0) {
        LayerDesc L{};
        L.kind = kind;
        L.cin = cin;
        L.cout = cout;
        L.stride = stride;
        L.ctx = ctx;
        L.ch = ctx ? cin - cout : 0;   // h has cout channels, z the rest
        n->layers.push_back(L);
    };
    add(L_CONV, 2, w[0], 1);
    for (int r = 0; r < n->down_res; ++r) add(L_CONV, w[0], w[0], 1), add(L_CONV, w[0], w[0], 1);
    for (int l = 1; l < 4; ++l) {
        add(L_CONV, w[l - 1], w[l], 2);
        for (int r = 0; r < n->down_res; ++r) add(L_CONV, w[l], w[l], 1), add(L_CONV, w[l], w[l], 1);
    }
    for (int l = 2; l >= 0; --l) {
        add(L_UP, w[l + 1], w[l], 2);
        add(L_CONV, 2 * w[l], w[l], 1);
        add(L_CONV, w[l], w[l], 1), add(L_CONV, w[l], w[l], 1);
    }
    n->n_enc = (int)n->layers.size();
    add(L_CONV, 2, w[0], 1);
    add(L_CONV, 2 * w[0], w[0], 1, 1);
    add(L_CONV, w[0], w[0], 1), add(L_CONV, w[0], w[0], 1);
    for (int l = 1; l < 4; ++l) {
        add(L_CONV, w[l - 1], w[l], 2);
        add(L_CONV, 2 * w[l], w[l], 1, 1);
        add(L_CONV, w[l], w[l], 1), add(L_CONV, w[l], w[l], 1);
    }
    for (int l = 2; l >= 0; --l) {
        add(L_UP, w[l + 1], w[l], 2);
        add(L_CONV, 2 * w[l], w[l], 1);
        add(L_CONV, w[l], w[l], 1), add(L_CONV, w[l], w[l], 1);
    }
    add(L_CONV, w[0], 2, 1);
    long o = 0, ob = 0;
    for (auto& L : n->layers) {
        L.nw = L.kind == L_CONV ? (long)L.cout * 9 * L.cin : 4L * L.cout * L.cin;
        L.woff = o;
        o += L.nw;
        L.boff = o;
        o += L.cout;
        if (L.kind == L_CONV) {
            L.K = pad32(9 * L.cin);
            L.Kt = pad32(9 * L.cout);
            L.wb_off = ob;
            ob += (long)L.cout * L.K;
            L.wt_off = ob;
            ob += (long)L.cin * L.Kt;
            if (L.ctx) {
                L.Kh = pad32(9 * L.ch);
                L.Kz = pad32(9 * (L.cin - L.ch));
                L.wh_off = ob;
                ob += (long)L.cout * L.Kh;
                L.wz_off = ob;
                ob += (long)L.cout * L.Kz;
            }
        } else {
            L.K = L.cin;
            L.Kt = 4 * L.cout;
            L.wb_off = ob;
            ob += 4L * L.cout * L.K;
            L.wt_off = ob;
            ob += (long)L.cin * L.Kt;
        }
    }
    n->nparam = o;
    n->nwb = ob;
}

// ------------------------------------------------------------------ elementwise kernels
// fp32 master -> bf16 forward copy [N][K] (zero padded) and data-gradient copy.
__global__ void k_refresh_conv(const float* __restrict__ W, int cout, int cin, int K, int Kt, bf16* __restrict__ wf,
                               bf16* __restrict__ wt) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nf = (long)cout * K;
    if (t < nf) {
        int co = (int)(t / K), k = (int)(t - (long)co * K);
        wf[t] = k < 9 * cin ? (bf16)W[(long)co * 9 * cin + k] : (bf16)0.0f;
    }
    long ntt = (long)cin * Kt;
    if (t < ntt) {
        // wt[ci][tap*cout + co] = W[co][tap][ci]
        int ci = (int)(t / Kt), k = (int)(t - (long)ci * Kt);
        bf16 v = (bf16)0.0f;
        if (k < 9 * cout) {
            int tap = k / cout, co = k - tap * cout;
            v = (bf16)W[((long)co * 9 + tap) * cin + ci];
        }
        wt[t] = v;
    }
}

// Split copies of a context convolution: wh[co][tap*ch + c] = W[co][tap][c],
// wz[co][tap*cz + c] = W[co][tap][ch + c] (zero padded to Kh, Kz).
__global__ void k_refresh_split(const float* __restrict__ W, int cout, int ch, int cz, int Kh, int Kz,
                                bf16* __restrict__ wh, bf16* __restrict__ wz) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int cin = ch + cz;
    if (t < (long)cout * Kh) {
        const int co = (int)(t / Kh), k = (int)(t - (long)co * Kh);
        bf16 v = (bf16)0.0f;
        if (k < 9 * ch) v = (bf16)W[((long)co * 9 + k / ch) * cin + k % ch];
        wh[t] = v;
    }
    if (t < (long)cout * Kz) {
        const int co = (int)(t / Kz), k = (int)(t - (long)co * Kz);
        bf16 v = (bf16)0.0f;
        if (k < 9 * cz) v = (bf16)W[((long)co * 9 + k / cz) * cin + ch + k % cz];
        wz[t] = v;
    }
}

__global__ void k_refresh_up(const float* __restrict__ W, int cout, int cin, bf16* __restrict__ wf,
                             bf16* __restrict__ wt) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long n = 4L * cout * cin;
    if (t >= n) return;
    wf[t] = (bf16)W[t];  // [ad][co][ci] == [n = ad*cout+co][k = ci]
    // wt[ci][ad*cout + co] = W[ad][co][ci]
    int ci = (int)(t / (4L * cout)), k = (int)(t - (long)ci * 4 * cout);
    wt[t] = (bf16)W[(long)k * cin + ci];
}

// Encoder input [omega^2 hx hz m, gamma] as bf16 [1][H][W][2].
__global__ void k_enc_input(const float* __restrict__ k2, const float* __restrict__ g, long n, float s,
                            bf16* __restrict__ out) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    out[2 * t] = (bf16)(s * k2[t]);
    out[2 * t + 1] = (bf16)g[t];
}

// Scaled residual input: out[b][p][0..1] = scale_b * (Re, Im) v_b[p].
template <typename T>
__global__ void k_pack(const cx<T>* __restrict__ v, long N, const double* __restrict__ sc, int scstride,
                       bf16* __restrict__ out, float* __restrict__ outf) {
    const int b = blockIdx.y;
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double s = sc[(long)b * scstride];
    cx<T> z = v[(long)b * N + p];
    float re = (float)(s * (double)z.re), im = (float)(s * (double)z.im);
    long o = ((long)b * N + p) * 2;
    out[o] = (bf16)re;
    out[o + 1] = (bf16)im;
    if (outf) {
        outf[o] = re;
        outf[o + 1] = im;
    }
}

// e_b = mul_b * (out[b][p][0] + i out[b][p][1]); e_b = 0 for a sample flagged
// in bad (non-finite network output), when bad is given.
template <typename T>
__global__ void k_unpack(const float* __restrict__ out, long N, const double* __restrict__ mul, int mstride,
                         const int* __restrict__ bad, cx<T>* __restrict__ e) {
    const int b = blockIdx.y;
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double m = mul[(long)b * mstride];
    if (bad && bad[b]) m = 0.0;
    long o = ((long)b * N + p) * 2;
    const float re = out[o], im = out[o + 1];
    e[(long)b * N + p] = m == 0.0 ? mk(T(0), T(0)) : mk(T(m * re), T(m * im));
}

__global__ void k_fill_int(int* __restrict__ a, int n, int v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// bad[b] = 1 when the network output of sample b holds a non-finite value
// (bad zeroed beforehand; one atomic per wave that sees one).
__global__ __launch_bounds__(256) void k_finite_flags(const float* __restrict__ out, long N,
                                                      const RhsState* __restrict__ st, int rhs0,
                                                      int* __restrict__ bad) {
    const int b = blockIdx.y;
    if (st) {
        const RhsState& S = st[rhs0 + b];
        if (!S.active || S.cycdone) return;
    }
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    bool nf = false;
    if (p < N) {
        const float2 v = reinterpret_cast<const float2*>(out)[(long)b * N + p];
        nf = !(__builtin_isfinite(v.x) && __builtin_isfinite(v.y));
    }
    if (__any(nf) && (threadIdx.x & 63) == 0) atomicOr(&bad[b], 1);
}

// Per-sample scale factors inside FGMRES: the raw basis vector V[j] enters with
// the normalisation v_j = vscale_j V[j], ||v_j|| = 1, and the preconditioner
// is applied to v_j: input multiplier s = sqrt(N) vscale_j, output multiplier
// hx hz / sqrt(N) (= hx hz ||v_j|| / sqrt(N)).
__global__ void k_scales_from_vscale(const double* __restrict__ vs, int stride, int nb, double sqrtN, double h2,
                                     double* __restrict__ s_in, double* __restrict__ s_out) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double v = vs[(long)b * stride];
    s_in[b] = sqrtN * v;
    s_out[b] = v > 0 ? h2 / sqrtN : 0.0;
}

// Per-sample 2-norm (deterministic block reduction), one block per sample;
// s_in = sqrt(N)/||r||, s_out = hx hz / s_in (0 for r = 0).
template <typename T>
__global__ __launch_bounds__(256) void k_sample_scale(const cx<T>* __restrict__ r, long N, double sqrtN, double h2,
                                                      double* __restrict__ s_in, double* __restrict__ s_out) {
    const int b = blockIdx.x;
    double acc = 0;
    for (long p = threadIdx.x; p < N; p += 256) acc += (double)norm2(r[(long)b * N + p]);
    acc = wave_sum(acc);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double nr = sqrt(ws[0] + ws[1] + ws[2] + ws[3]);
        s_in[b] = nr > 0 ? sqrtN / nr : 0.0;
        s_out[b] = nr > 0 ? h2 * nr / sqrtN : 0.0;
    }
}

// Masked gradient of a ReLU output: gm = bf16(g * (y > 0)) (or g if no activation).
__global__ void k_relu_bwd(const float* __restrict__ g, const bf16* __restrict__ y, long n, int act,
                           bf16* __restrict__ gm) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float v = g[t];
    if (act && !((float)y[t] > 0.f)) v = 0.f;
    gm[t] = (bf16)v;
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, bf16* __restrict__ b, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (bf16)a[t];
}

__global__ void k_axpy_f32(const float* __restrict__ x, float* __restrict__ y, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += x[t];
}

// y[p] += sum_b x[b][p]   (broadcast context gradient, fixed order)
__global__ void k_batch_sum(const float* __restrict__ x, int B, long n, float* __restrict__ y) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float s = 0;
    for (int b = 0; b < B; ++b) s += x[(long)b * n + t];
    y[t] += s;
}

// Bias gradient partials: part[blk][c] = sum over the block's pixels of gm[p][c].
// The block reads a contiguous run of the flat [P][C] array in steps of
// `stride` elements (the largest multiple of lcm(8, C) up to 2048), 8 elements
// per lane, so a lane's elements keep their channels from step to step; the
// lane sums are then folded per channel in LDS in a fixed order.
constexpr int BIAS_STEPS = 32;           // steps per block
__global__ __launch_bounds__(256) void k_bias_part(const bf16* __restrict__ gm, long n, int C, int stride,
                                                   float* __restrict__ part) {
    __shared__ float red[2048];
    __shared__ float red2[256];
    const int tid = threadIdx.x;
    const long q0 = (long)blockIdx.x * BIAS_STEPS * stride;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (8 * tid < stride) {
        for (int it = 0; it < BIAS_STEPS; ++it) {
            const long q = q0 + (long)it * stride + 8 * tid;
            if (q + 8 <= n) {
                bf16x8 v = *reinterpret_cast<const bf16x8*>(gm + q);
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[e] += (float)v[e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (q + e < n) acc[e] += (float)gm[q + e];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[8 * tid + e] = acc[e];
    __syncthreads();
    const int units = stride / C;
    if (C <= 256) {
        const int G = 256 / C;           // lanes per channel
        if (tid < G * C) {
            const int c = tid % C, g = tid / C;
            float v = 0;
            for (int j = g; j < units; j += G) v += red[c + j * C];
            red2[tid] = v;
        }
        __syncthreads();
        if (tid < C) {
            float v = 0;
            for (int g = 0; g < G; ++g) v += red2[g * C + tid];
            part[(long)blockIdx.x * C + tid] = v;
        }
    } else {
        for (int c = tid; c < C; c += 256) {
            float v = 0;
            for (int j = 0; j < units; ++j) v += red[c + j * C];
            part[(long)blockIdx.x * C + c] = v;
        }
    }
}

// out[c] += sum_q part[q][c]: one block per column, fixed-order tree in LDS.
__global__ __launch_bounds__(256) void k_fold_cols(const float* __restrict__ part, int nq, int C,
                                                   float* __restrict__ out) {
    __shared__ float red[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    float s = 0;
    for (int q = tid; q < nq; q += 256) s += part[(long)q * C + c];
    red[tid] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) out[c] += red[0];
}

// out[i] (+)= sum_s part[s][i]  (fixed order over the splits)
__global__ void k_sum_splits(const float* __restrict__ part, int nsplit, long n, long stride, int accumulate,
                             float* __restrict__ out) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float s = 0;
    for (int q = 0; q < nsplit; ++q) s += part[(long)q * stride + t];
    out[t] = accumulate ? out[t] + s : s;
}

// dW[row][col] += sum_s part[s][row][col] for col < N (rows of Npad columns);
// four interleaved partial sums (fixed order) keep several loads in flight.
__global__ void k_sum_wsplits(const float* __restrict__ part, int nsplit, int M, int N, int Npad,
                              float* __restrict__ out) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)M * N) return;
    int row = (int)(t / N), col = (int)(t - (long)row * N);
    const long stride = (long)M * Npad;
    const float* p = part + (long)row * Npad + col;
    float s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int q = 0;
    for (; q + 4 <= nsplit; q += 4) {
        s0 += p[(long)q * stride];
        s1 += p[(long)(q + 1) * stride];
        s2 += p[(long)(q + 2) * stride];
        s3 += p[(long)(q + 3) * stride];
    }
    for (; q < nsplit; ++q) s0 += p[(long)q * stride];
    out[t] += (s0 + s1) + (s2 + s3);
}

// MSE: d = out - tgt; grad = 2 d / B; per-block partial of sum d^2.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ tgt, long n,
                                             float inv_b, float* __restrict__ grad, double* __restrict__ part) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0;
    if (t < n) {
        float d = out[t] - tgt[t];
        grad[t] = 2.f * d * inv_b;
        s = (double)d * d;
    }
    s = wave_sum(s);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Target s e / (hx hz) as fp32 [B][N][2].
__global__ void k_target(const c64* __restrict__ e, long N, const double* __restrict__ s_in, double inv_h2,
                         float* __restrict__ tgt) {
    const int b = blockIdx.y;
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double s = s_in[b] * inv_h2;
    c64 z = e[(long)b * N + p];
    tgt[((long)b * N + p) * 2] = (float)(s * z.re);
    tgt[((long)b * N + p) * 2 + 1] = (float)(s * z.im);
}

// Adam on the fp32 master weights (bias-corrected), zeroes the gradient.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float gt = g[t];
    float mt = b1 * m[t] + (1.f - b1) * gt;
    float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    float mh = mt / c1, vh = vt / c2;
    w[t] -= lr * mh / (sqrtf(vh) + eps);
    g[t] = 0.f;
}

// Complex normal x_i ~ CN(0,1) from Philox: counter (p, stream i), key (seed, 0xDA7A).
__global__ void k_randn_c(c128* __restrict__ x, long N, int first, uint32_t seed) {
    const int b = blockIdx.y;
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    u32x4 w = philox_at((uint64_t)p, (uint32_t)(first + b), seed, 0xDA7Au);
    double u0 = philox_u01(w.v[0]), u1 = philox_u01(w.v[1]);
    double rad = sqrt(-2.0 * log(u0)) * sqrt(0.5);
    double ang = 2.0 * M_PI * u1;
    x[(long)b * N + p] = mk(rad * cos(ang), rad * sin(ang));
}

__global__ void k_c128_to_c64(const c128* __restrict__ a, c64* __restrict__ b, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = ccast<float>(a[t]);
}
__global__ void k_c64_to_c128(const c64* __restrict__ a, c128* __restrict__ b, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = ccast<double>(a[t]);
}
__global__ void k_sub_c128(const c128* __restrict__ a, const c128* __restrict__ b, c128* __restrict__ out, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = a[t] - b[t];
}

static dim3 g1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// ------------------------------------------------------------------ activation arena
struct Tens {
    int B = 0, H = 0, W = 0, C = 0;
    bf16* d = nullptr;
    float* g = nullptr;  // gradient (training only)
    long n() const { return (long)B * H * W * C; }
    long bs() const { return (long)H * W * C; }
};

enum { OP_CONV = 0, OP_UP = 1 };
struct Op {
    int kind, layer, in1, in2, out, stride, relu, resid;
    bool bcast2;  // in2 is the broadcast context (batch 1)
};

struct Program {
    std::vector<Tens> t;
    std::vector<Op> ops;
    int input = -1, output = -1;
    int z[4] = {-1, -1, -1, -1};
    float* outf = nullptr;  // fp32 copy of the final output (solver)
};

// Encoder outputs of one operator for one network version (inference): the
// context maps z_0..z_3 and the z parts of the solver's context convolutions.
// Kept per operator, so a batch that alternates between operators of one grid
// does not re-run the encoder.
struct EncCtx {
    uint64_t net_uid = 0, ver = 0;
    Tens zt[4];              // batch-1 views of z_l
    bf16* zc[4] = {nullptr, nullptr, nullptr, nullptr};   // z parts of the context convolutions (+ bias)
    std::vector<void*> allocs;
    ~EncCtx() {
        for (void* p : allocs) (void)hipFree(p);
    }
};

struct Arena {
    int B = 0, H = 0, W = 0;
    bool train = false;
    const EncCtx* ctx = nullptr;   // inference: context of the operator being applied
    Program enc, sol;
    std::vector<void*> allocs;
    float* work = nullptr;   // wgrad / bias partials
    size_t work_elems = 0;
    float* zg[4] = {nullptr, nullptr, nullptr, nullptr};  // per-sample context gradients
    bf16* gm = nullptr;      // masked output gradient (bf16), largest tensor
    ~Arena() {
        for (void* p : allocs) (void)hipFree(p);
    }
};

static int dalloc(Arena& A, void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
        return fail(HELM_ENOMEM, "cnn: hipMalloc(%zu) failed", bytes);
    A.allocs.push_back(*p);
    return HELM_OK;
}

static int new_tensor(Program& P, int B, int H, int W, int C) {
    Tens t;
    t.B = B;
    t.H = H;
    t.W = W;
    t.C = C;
    P.t.push_back(t);
    return (int)P.t.size() - 1;
}

// Builds the forward programs (tensor shapes and op list) of both networks.
static void build_programs(const cnn_net* net, Arena& A) {
    const int* w = net->widths;
    int H = A.H, W = A.W;
    Program& E = A.enc;
    int li = 0;
    auto conv = [&](Program& P, int in1, int in2, int cout, int stride, int relu, int resid, bool bc) {
        const Tens& x = P.t[in1];
        int Ho = (x.H + stride - 1) / stride, Wo = (x.W + stride - 1) / stride;
        int o = new_tensor(P, x.B, Ho, Wo, cout);
        P.ops.push_back({OP_CONV, li++, in1, in2, o, stride, relu, resid, bc});
        return o;
    };
    auto up = [&](Program& P, int in, int cout) {
        const Tens& x = P.t[in];
        int o = new_tensor(P, x.B, 2 * x.H, 2 * x.W, cout);
        P.ops.push_back({OP_UP, li++, in, -1, o, 2, 1, -1, false});
        return o;
    };
    auto res = [&](Program& P, int x) {
        int h = conv(P, x, -1, P.t[x].C, 1, 1, -1, false);
        return conv(P, h, -1, P.t[x].C, 1, 0, x, false);
    };
    E.input = new_tensor(E, 1, H, W, 2);
    int h = conv(E, E.input, -1, w[0], 1, 1, -1, false);
    for (int r = 0; r < net->down_res; ++r) h = res(E, h);
    int skip[4];
    skip[0] = h;
    for (int l = 1; l < 4; ++l) {
        h = conv(E, h, -1, w[l], 2, 1, -1, false);
        for (int r = 0; r < net->down_res; ++r) h = res(E, h);
        skip[l] = h;
    }
    E.z[3] = h;
    for (int l = 2; l >= 0; --l) {
        int u = up(E, h, w[l]);
        h = conv(E, u, skip[l], w[l], 1, 1, -1, false);
        h = res(E, h);
        E.z[l] = h;
    }
    // solver
    Program& S = A.sol;
    S.input = new_tensor(S, A.B, H, W, 2);
    // the context tensors live in the encoder program; the solver refers to them
    // through ids -(l+2) (-1 means "no second source")
    h = conv(S, S.input, -1, w[0], 1, 1, -1, false);
    for (int l = 0; l < 4; ++l) {
        if (l > 0) h = conv(S, h, -1, w[l], 2, 1, -1, false);
        h = conv(S, h, -(l + 2), w[l], 1, 1, -1, true);
        h = res(S, h);
        skip[l] = h;
    }
    for (int l = 2; l >= 0; --l) {
        int u = up(S, h, w[l]);
        h = conv(S, u, skip[l], w[l], 1, 1, -1, false);
        h = res(S, h);
    }
    S.output = conv(S, h, -1, 2, 1, 0, -1, false);
}

static int alloc_arena(const cnn_net* net, Arena& A) {
    build_programs(net, A);
    int rc;
    for (Program* P : {&A.enc, &A.sol}) {
        for (auto& t : P->t) {
            if ((rc = dalloc(A, (void**)&t.d, sizeof(bf16) * t.n()))) return rc;
            if (A.train && (rc = dalloc(A, (void**)&t.g, sizeof(float) * t.n()))) return rc;
        }
    }
    if ((rc = dalloc(A, (void**)&A.sol.outf, sizeof(float) * A.sol.t[A.sol.output].n()))) return rc;
    if (A.train) {
        for (int l = 0; l < 4; ++l) {
            const Tens& z = A.enc.t[A.enc.z[l]];
            if ((rc = dalloc(A, (void**)&A.zg[l], sizeof(float) * z.n() * A.B))) return rc;
        }
        // partial sums of the weight gradients: nsplit x M x Npad
        size_t mx = 0;
        for (const auto& L : net->layers) {
            size_t m = L.kind == L_CONV ? L.cout : 4 * L.cout;
            size_t n = L.kind == L_CONV ? 9 * L.cin : L.cin;
            mx = std::max(mx, m * ((n + 63) / 64 * 64));
        }
        A.work_elems = mx * 64;
        if ((rc = dalloc(A, (void**)&A.work, sizeof(float) * A.work_elems))) return rc;
        size_t mt = 0;
        for (Program* P : {&A.enc, &A.sol})
            for (auto& t : P->t) mt = std::max(mt, (size_t)t.n());
        if ((rc = dalloc(A, (void**)&A.gm, sizeof(bf16) * mt))) return rc;
    }
    return HELM_OK;
}

// ------------------------------------------------------------------ forward / backward
static const Tens& tens_of(const Arena& A, const Program& P, int id) {
    if (id <= -2) return A.ctx ? A.ctx->zt[-id - 2] : A.enc.t[A.enc.z[-id - 2]];
    return P.t[id];
}

// Ops oi, oi+1 form a 32-channel residual block y = x + conv(ReLU(conv(x))) that
// inference runs as one fused kernel (the intermediate stays in LDS).
static bool fusable_resblock(const cnn_net* net, const Arena& A, const Program& P, size_t oi) {
    if (A.train || oi + 1 >= P.ops.size()) return false;
    const Op& a = P.ops[oi];
    const Op& b = P.ops[oi + 1];
    if (a.kind != OP_CONV || b.kind != OP_CONV || a.stride != 1 || b.stride != 1) return false;
    if (!a.relu || b.relu || a.resid >= 0 || a.in2 != -1 || b.in2 != -1) return false;
    if (b.in1 != a.out || b.resid != a.in1 || a.in1 < 0) return false;
    const Tens& x = P.t[a.in1];
    const Tens& h = P.t[a.out];
    const Tens& y = P.t[b.out];
    return x.C == 32 && h.C == 32 && y.C == 32 && net->layers[a.layer].K >= 288 && net->layers[b.layer].K >= 288;
}

// The solver's first layer (2 -> 32 channels) followed by the level-0 context
// convolution in its split form, with nothing else reading the first layer's
// output: one fused kernel at inference.
static bool fusable_first_ctx(const cnn_net* net, const Arena& A, const Program& P, size_t oi) {
    if (A.train || !A.ctx || oi + 1 >= P.ops.size()) return false;
    const Op& a = P.ops[oi];
    const Op& b = P.ops[oi + 1];
    if (a.kind != OP_CONV || b.kind != OP_CONV || a.stride != 1 || b.stride != 1) return false;
    if (!a.relu || !b.relu || a.resid >= 0 || b.resid >= 0 || a.in2 != -1 || b.in1 != a.out || b.out == P.output)
        return false;
    const LayerDesc& Lb = net->layers[b.layer];
    if (!(Lb.ctx && b.bcast2 && b.in2 <= -2)) return false;
    for (size_t j = oi + 2; j < P.ops.size(); ++j) {
        const Op& o = P.ops[j];
        if (o.in1 == a.out || o.in2 == a.out || o.resid == a.out) return false;
    }
    const Tens& x = tens_of(A, P, a.in1);
    const Tens& h = P.t[a.out];
    const Tens& y = P.t[b.out];
    return x.C == 2 && h.C == 32 && y.C == 32 && x.H == y.H && x.W == y.W && x.B == y.B &&
           net->layers[a.layer].K >= 32 && Lb.Kh >= 288;
}

static int run_forward(const cnn_net* net, Arena& A, Program& P, const RhsState* st, int rhs0, hipStream_t s) {
    for (size_t oi = 0; oi < P.ops.size(); ++oi) {
        const Op& op = P.ops[oi];
        if (fusable_first_ctx(net, A, P, oi)) {
            const Op& o2 = P.ops[oi + 1];
            const LayerDesc& L0 = net->layers[op.layer];
            const LayerDesc& L1 = net->layers[o2.layer];
            const Tens& x = tens_of(A, P, op.in1);
            FirstCtxArgs f{};
            f.r = x.d;
            f.B = x.B;
            f.H = x.H;
            f.W = x.W;
            f.w0 = net->wb + L0.wb_off;
            f.K0 = L0.K;
            f.b0 = net->master + L0.boff;
            f.wh = net->wb + L1.wh_off;
            f.Kh = L1.Kh;
            f.bmap = A.ctx->zc[-o2.in2 - 2];
            f.out = P.t[o2.out].d;
            f.st = (&P == &A.sol) ? st : nullptr;
            f.rhs0 = rhs0;
            int rc = launch_first_ctx(f, s);
            if (rc) return rc;
            ++oi;
            continue;
        }
        if (fusable_resblock(net, A, P, oi)) {
            const Op& o2 = P.ops[oi + 1];
            const LayerDesc& L1 = net->layers[op.layer];
            const LayerDesc& L2 = net->layers[o2.layer];
            const Tens& x = P.t[op.in1];
            ResArgs r{};
            r.x = x.d;
            r.B = x.B;
            r.H = x.H;
            r.W = x.W;
            r.w1 = net->wb + L1.wb_off;
            r.K1 = L1.K;
            r.b1 = net->master + L1.boff;
            r.w2 = net->wb + L2.wb_off;
            r.K2 = L2.K;
            r.b2 = net->master + L2.boff;
            r.out = P.t[o2.out].d;
            r.st = (&P == &A.sol) ? st : nullptr;
            r.rhs0 = rhs0;
            int rc = launch_resblock32(r, s);
            if (rc) return rc;
            ++oi;
            continue;
        }
        const LayerDesc& L = net->layers[op.layer];
        const Tens& x = tens_of(A, P, op.in1);
        Tens& y = P.t[op.out];
        GemmArgs g{};
        g.a1 = x.d;
        g.c1 = x.C;
        g.abs1 = x.bs();
        g.B = y.B;
        g.Hi = x.H;
        g.Wi = x.W;
        g.stride = op.stride;
        g.w = net->wb + L.wb_off;
        g.K = L.K;
        g.bias = net->master + L.boff;
        g.relu = op.relu;
        g.out = y.d;
        g.st = (&P == &A.sol) ? st : nullptr;
        g.rhs0 = rhs0;
        const bool split = L.ctx && A.ctx && op.bcast2 && op.in2 <= -2;
        if (op.in2 != -1 && !split) {
            const Tens& x2 = tens_of(A, P, op.in2);
            g.a2 = x2.d;
            g.c2 = x2.C;
            g.abs2 = op.bcast2 ? 0 : x2.bs();
        }
        if (split) {
            // conv(concat(h, z)) = conv_h(h) + [conv_z(z) + b], the bracket precomputed per encoder pass
            g.w = net->wb + L.wh_off;
            g.K = L.Kh;
            g.bmap = A.ctx->zc[-op.in2 - 2];
        }
        if (op.kind == OP_CONV) {
            g.gmode = G_CONV;
            g.Ho = y.H;
            g.Wo = y.W;
            g.N = y.C;
            g.kvalid = 9 * (g.c1 + g.c2);
            g.epi = E_FWD;
            g.resid = op.resid >= 0 ? P.t[op.resid].d : nullptr;
            g.outf = op.out == P.output ? P.outf : nullptr;
            g.M = (long)y.B * y.H * y.W;
        } else {
            g.gmode = G_UP;
            g.Ho = x.H;
            g.Wo = x.W;
            g.N = 4 * y.C;
            g.kvalid = x.C;
            g.epi = E_UPFWD;
            g.M = (long)x.B * x.H * x.W;
        }
        int rc = launch_gemm(g, s);
        if (rc) return rc;
    }
    return HELM_OK;
}

// db[c] += sum over pixels of gm[p][c] (gm flat [n / C][C]).
static int bias_grad(const bf16* gm, long n, int C, float* work, size_t work_elems, float* db, hipStream_t s) {
    long l = C;
    while (l % 8) l += C;                // lcm(8, C)
    if (C <= 0 || l > 2048) return fail(HELM_EINVAL, "cnn: bias gradient of %d channels unsupported", C);
    const int stride = (int)(2048 / l * l);
    const int nb = (int)((n + (long)BIAS_STEPS * stride - 1) / ((long)BIAS_STEPS * stride));
    if ((size_t)nb * C > work_elems) return fail(HELM_EINVAL, "cnn: bias scratch too small");
    if (nb == 0) return HELM_OK;
    hipLaunchKernelGGL(k_bias_part, dim3(nb), dim3(256), 0, s, gm, n, C, stride, work);
    HELM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_fold_cols, dim3(C), dim3(256), 0, s, work, nb, C, db);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

// Backward through a program.  Gradients of tensors are fp32 and must be zero
// on entry except the seeded output gradient; parameter gradients accumulate
// into net->grad.  Context gradients (solver -> encoder) go to A.zg (per sample).
static int run_backward(cnn_net* net, Arena& A, Program& P, hipStream_t s) {
    int rc;
    bf16* gm = A.gm;
    for (int oi = (int)P.ops.size() - 1; oi >= 0; --oi) {
        const Op& op = P.ops[oi];
        const LayerDesc& L = net->layers[op.layer];
        Tens& y = P.t[op.out];
        const Tens& x = tens_of(A, P, op.in1);
        const long ny = y.n();
        hipLaunchKernelGGL(k_relu_bwd, g1(ny), dim3(256), 0, s, y.g, y.d, ny, op.relu, gm);
        HELM_CHECK_LAUNCH();
        if (op.resid >= 0) {
            hipLaunchKernelGGL(k_axpy_f32, g1(ny), dim3(256), 0, s, y.g, P.t[op.resid].g, ny);
            HELM_CHECK_LAUNCH();
        }
        // bias gradient
        {
            if ((rc = bias_grad(gm, y.n(), y.C, A.work, A.work_elems, net->grad + L.boff, s))) return rc;
        }
        // weight gradient
        {
            WgradArgs w{};
            w.g = gm;
            w.Hg = y.H;
            w.Wg = y.W;
            w.Cg = y.C;
            w.a1 = x.d;
            w.c1 = x.C;
            w.abs1 = x.bs();
            w.B = y.B;
            w.Hi = x.H;
            w.Wi = x.W;
            w.stride = op.stride;
            if (op.in2 != -1) {
                const Tens& x2 = tens_of(A, P, op.in2);
                w.a2 = x2.d;
                w.c2 = x2.C;
                w.abs2 = op.bcast2 ? 0 : x2.bs();
            }
            if (op.kind == OP_CONV) {
                w.mode = G_CONV;
                w.M = y.C;
                w.N = 9 * (w.c1 + w.c2);
                w.P = (long)y.B * y.H * y.W;
            } else {
                w.mode = G_UP;
                w.M = 4 * y.C;
                w.N = x.C;
                w.P = (long)x.B * x.H * x.W;
            }
            w.Npad = (w.N + 63) / 64 * 64;
            w.part = A.work;
            int nsplit = 0;
            if ((rc = launch_wgrad(w, (int)(A.work_elems / ((size_t)w.M * w.Npad)), s, &nsplit))) return rc;
            long nw = (long)w.M * w.N;
            hipLaunchKernelGGL(k_sum_wsplits, g1(nw), dim3(256), 0, s, A.work, nsplit, w.M, w.N, w.Npad,
                               net->grad + L.woff);
            HELM_CHECK_LAUNCH();
        }
        // data gradient (not needed for the network inputs)
        const bool need_x = !(op.in1 == P.input && op.in2 == -1);
        if (!need_x) continue;
        GemmArgs g{};
        g.a1 = gm;
        g.c1 = y.C;
        g.abs1 = y.bs();
        g.B = y.B;
        g.Hi = y.H;
        g.Wi = y.W;
        g.stride = op.stride;
        g.w = net->wb + L.wt_off;
        g.K = L.Kt;
        g.epi = E_ACC;
        g.Ho = x.H;
        g.Wo = x.W;
        g.M = (long)y.B * x.H * x.W;
        g.acc1 = x.g;
        g.n1 = x.C;
        if (op.kind == OP_CONV) {
            g.gmode = G_CONVT;
            g.kvalid = 9 * y.C;
            int c2 = 0;
            if (op.in2 != -1) {
                const Tens& x2 = tens_of(A, P, op.in2);
                c2 = x2.C;
                g.acc2 = op.in2 <= -2 ? A.zg[-op.in2 - 2] : x2.g;
            }
            g.N = x.C + c2;
        } else {
            g.gmode = G_UPT;
            g.kvalid = 4 * y.C;
            g.N = x.C;
        }
        if ((rc = launch_gemm(g, s))) return rc;
    }
    return HELM_OK;
}

// ------------------------------------------------------------------ arenas and encoder cache
struct NetState {
    std::map<std::tuple<int, int, int, int, int>, Arena*> arenas;  // (B, H, W, train, slot)
};
static std::map<const cnn_net*, NetState> g_state;
static std::recursive_mutex g_cnn_mutex;

// slot tells apart arenas of the same shape that are in use at the same time
// (the two halves of a batch applied on two streams).
static int get_arena(cnn_net* net, int B, int H, int W, bool train, Arena** out, int slot = 0) {
    auto& ns = g_state[net];
    auto key = std::make_tuple(B, H, W, (int)train, slot);
    auto it = ns.arenas.find(key);
    if (it != ns.arenas.end()) {
        *out = it->second;
        return HELM_OK;
    }
    Arena* A = new Arena();
    A->B = B;
    A->H = H;
    A->W = W;
    A->train = train;
    int rc = alloc_arena(net, *A);
    if (rc) {
        delete A;
        return rc;
    }
    ns.arenas[key] = A;
    *out = A;
    return HELM_OK;
}

static int refresh_weights(cnn_net* net, hipStream_t s) {
    for (const auto& L : net->layers) {
        if (L.kind == L_CONV) {
            long n = std::max<long>((long)L.cout * L.K, (long)L.cin * L.Kt);
            hipLaunchKernelGGL(k_refresh_conv, g1(n), dim3(256), 0, s, net->master + L.woff, L.cout, L.cin, L.K, L.Kt,
                               net->wb + L.wb_off, net->wb + L.wt_off);
            if (L.ctx) {
                HELM_CHECK_LAUNCH();
                long ns = (long)L.cout * std::max(L.Kh, L.Kz);
                hipLaunchKernelGGL(k_refresh_split, g1(ns), dim3(256), 0, s, net->master + L.woff, L.cout, L.ch,
                                   L.cin - L.ch, L.Kh, L.Kz, net->wb + L.wh_off, net->wb + L.wz_off);
            }
        } else {
            hipLaunchKernelGGL(k_refresh_up, g1(4L * L.cout * L.cin), dim3(256), 0, s, net->master + L.woff, L.cout,
                               L.cin, net->wb + L.wb_off, net->wb + L.wt_off);
        }
        HELM_CHECK_LAUNCH();
    }
    net->version++;
    return HELM_OK;
}

static int check_grid(const helm_op* op) {
    if (op->nz % 8 || op->nx % 8) return fail(HELM_EINVAL, "cnn: grid %d x %d must be divisible by 8", op->nz, op->nx);
    return HELM_OK;
}

// Encoder pass for (net, op) into the arena's encoder program.
static int encode(cnn_net* net, const helm_op* op, Arena& A, hipStream_t s, EncCtx* ctx = nullptr) {
    long n = op->n();
    float sc = (float)(op->omega * op->omega * op->hx * op->hz);
    hipLaunchKernelGGL(k_enc_input, g1(n), dim3(256), 0, s, op->lv[0].k2, op->lv[0].g, n, sc,
                       A.enc.t[A.enc.input].d);
    HELM_CHECK_LAUNCH();
    A.ctx = nullptr;
    int rc = run_forward(net, A, A.enc, nullptr, 0, s);
    if (rc || !ctx) return rc;
    for (int l = 0; l < 4; ++l) {
        const Tens& z = A.enc.t[A.enc.z[l]];
        HELM_HIP(hipMemcpyAsync(ctx->zt[l].d, z.d, sizeof(bf16) * z.n(), hipMemcpyDeviceToDevice, s));
    }
    // z parts of the solver's context convolutions (batch independent)
    for (const Op& o : A.sol.ops) {
        const LayerDesc& L = net->layers[o.layer];
        if (!L.ctx || o.in2 > -2) continue;
        const int l = -o.in2 - 2;
        const Tens& z = ctx->zt[l];
        GemmArgs g{};
        g.gmode = G_CONV;
        g.a1 = z.d;
        g.c1 = z.C;
        g.abs1 = z.bs();
        g.B = 1;
        g.Hi = z.H;
        g.Wi = z.W;
        g.Ho = z.H;
        g.Wo = z.W;
        g.stride = 1;
        g.w = net->wb + L.wz_off;
        g.K = L.Kz;
        g.kvalid = 9 * z.C;
        g.N = L.cout;
        g.epi = E_FWD;
        g.bias = net->master + L.boff;
        g.relu = 0;
        g.out = ctx->zc[l];
        g.M = (long)z.H * z.W;
        if ((rc = launch_gemm(g, s))) return rc;
    }
    return HELM_OK;
}


// Makes A->ctx the encoder context of (net, op), running the encoder only when
// the operator has none for this network version.
static int ensure_encoded(cnn_net* net, const helm_op* op, Arena* A, hipStream_t s) {
    EncCtx* ctx = (EncCtx*)op->enc.ctx;
    if (ctx && ctx->net_uid == net->uid && ctx->ver == net->version) {
        A->ctx = ctx;
        return HELM_OK;
    }
    if (!ctx) {
        ctx = new EncCtx();
        for (int l = 0; l < 4; ++l) {
            Tens t = A->enc.t[A->enc.z[l]];
            t.g = nullptr;
            void* p = nullptr;
            if (hipMalloc(&p, sizeof(bf16) * t.n()) != hipSuccess) {
                delete ctx;
                return fail(HELM_ENOMEM, "cnn: encoder context");
            }
            ctx->allocs.push_back(p);
            t.d = (bf16*)p;
            ctx->zt[l] = t;
            if (hipMalloc(&p, sizeof(bf16) * t.n()) != hipSuccess) {
                delete ctx;
                return fail(HELM_ENOMEM, "cnn: encoder context");
            }
            ctx->allocs.push_back(p);
            ctx->zc[l] = (bf16*)p;
        }
        const_cast<helm_op*>(op)->enc.ctx = ctx;
    }
    ctx->net_uid = 0;
    int rc = encode(net, op, *A, s, ctx);
    if (rc) return rc;
    ctx->net_uid = net->uid;
    ctx->ver = net->version;
    A->ctx = ctx;
    return HELM_OK;
}

void cnn_release_cache(helm_op* op) {
    delete (EncCtx*)op->enc.ctx;
    op->enc.ctx = nullptr;
}

// Per-batch-size scale buffers (s_in, s_out per RHS) and the per-RHS flags of
// non-finite network outputs, allocated once.
struct ScaleBufs {
    double* sin = nullptr;
    double* sout = nullptr;
    int* bad = nullptr;
};
static int scale_bufs(int nrhs, ScaleBufs* out, int slot = 0) {
    static std::map<std::pair<int, int>, ScaleBufs> sbuf;
    auto& sb = sbuf[{nrhs, slot}];
    if (!sb.sin) {
        if (hipMalloc(&sb.sin, sizeof(double) * nrhs) != hipSuccess ||
            hipMalloc(&sb.sout, sizeof(double) * nrhs) != hipSuccess ||
            hipMalloc(&sb.bad, sizeof(int) * nrhs) != hipSuccess)
            return fail(HELM_ENOMEM, "cnn: scale buffers");
    }
    *out = sb;
    return HELM_OK;
}

// Everything a preconditioner application for nrhs right-hand sides of op
// allocates or computes once (arena, encoder context, scale buffers), done
// eagerly so that later applications can be captured into a graph.
int cnn_prepare(cnn_net* net, const helm_op* op, int nrhs, hipStream_t s, int slot) {
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    int rc;
    if ((rc = check_grid(op))) return rc;
    Arena* A;
    if ((rc = get_arena(net, nrhs, op->nz, op->nx, false, &A, slot))) return rc;
    if ((rc = ensure_encoded(net, op, A, s))) return rc;
    ScaleBufs sb;
    return scale_bufs(nrhs, &sb, slot);
}

// e = M_net(r) for nrhs vectors.  Scales: s_in = sqrt(N) fscale (FGMRES basis
// vectors have unit norm after scaling) or sqrt(N)/||r|| when fscale is null.
// With fallback, a right-hand side whose network output holds a non-finite
// value gets e = 0 instead (inside M_VU that leaves the V-cycle alone for it).
template <typename T>
static int apply_impl(cnn_net* net, const helm_op* op, const cx<T>* r, const double* fscale, int fstride, cx<T>* e,
                      int nrhs, const RhsState* st, int rhs0, hipStream_t s, bool fallback = false, int slot = 0) {
    int rc;
    if ((rc = check_grid(op))) return rc;
    Arena* A;
    if ((rc = get_arena(net, nrhs, op->nz, op->nx, false, &A, slot))) return rc;
    if ((rc = ensure_encoded(net, op, A, s))) return rc;
    ScaleBufs sb;
    if ((rc = scale_bufs(nrhs, &sb, slot))) return rc;
    const long N = op->n();
    const double sqrtN = std::sqrt((double)N), h2 = op->hx * op->hz;
    if (fscale) {
        hipLaunchKernelGGL(k_scales_from_vscale, dim3((nrhs + 63) / 64), dim3(64), 0, s, fscale + (long)rhs0 * fstride,
                           fstride, nrhs, sqrtN, h2, sb.sin, sb.sout);
    } else {
        hipLaunchKernelGGL(k_sample_scale<T>, dim3(nrhs), dim3(256), 0, s, r, N, sqrtN, h2, sb.sin, sb.sout);
    }
    HELM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, s, r, N, sb.sin, 1,
                       A->sol.t[A->sol.input].d, (float*)nullptr);
    HELM_CHECK_LAUNCH();
    if ((rc = run_forward(net, *A, A->sol, st, rhs0, s))) return rc;
    const dim3 grid((unsigned)((N + 255) / 256), nrhs);
    if (fallback) {
        // a fill kernel, not a memset, so that the step can be graph-captured
        hipLaunchKernelGGL(k_fill_int, dim3((nrhs + 255) / 256), dim3(256), 0, s, sb.bad, nrhs, 0);
        HELM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_finite_flags, grid, dim3(256), 0, s, A->sol.outf, N, st, rhs0, sb.bad);
        HELM_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_unpack<T>, grid, dim3(256), 0, s, A->sol.outf, N, sb.sout, 1,
                       fallback ? (const int*)sb.bad : nullptr, e);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

int cnn_apply_masked(cnn_net* net, const helm_op* op, const void* r, const double* fscale, int fstride, void* e,
                     int nrhs, const RhsState* st, int rhs0, int wide, hipStream_t s, bool fallback, int slot) {
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    // fscale arrives offset to the current Arnoldi column; apply_impl adds rhs0*stride
    if (wide)
        return apply_impl<double>(net, op, (const c128*)r, fscale, fstride, (c128*)e, nrhs, st, rhs0, s, fallback,
                                  slot);
    return apply_impl<float>(net, op, (const c64*)r, fscale, fstride, (c64*)e, nrhs, st, rhs0, s, fallback, slot);
}

// ------------------------------------------------------------------ training
static int zero_grads(Arena& A, hipStream_t s) {
    for (Program* P : {&A.enc, &A.sol})
        for (auto& t : P->t) HELM_HIP(hipMemsetAsync(t.g, 0, sizeof(float) * t.n(), s));
    for (int l = 0; l < 4; ++l) {
        const Tens& z = A.enc.t[A.enc.z[l]];
        HELM_HIP(hipMemsetAsync(A.zg[l], 0, sizeof(float) * z.n() * A.B, s));
    }
    return HELM_OK;
}

// Loss and parameter gradient (accumulated into net->grad) of one batch of
// (r, e) pairs (c64, back to back).  Returns the loss on the host.
static int loss_grad(cnn_net* net, const helm_op* op, const c64* r, const c64* e, int B, double* loss,
                     hipStream_t s) {
    int rc;
    if ((rc = check_grid(op))) return rc;
    Arena* A;
    if ((rc = get_arena(net, B, op->nz, op->nx, true, &A))) return rc;
    if ((rc = zero_grads(*A, s))) return rc;
    if ((rc = encode(net, op, *A, s))) return rc;
    const long N = op->n();
    const double sqrtN = std::sqrt((double)N), h2 = op->hx * op->hz;
    static std::map<int, std::pair<double*, double*>> sbuf;
    auto& sb = sbuf[B];
    if (!sb.first) {
        if (hipMalloc(&sb.first, sizeof(double) * B) != hipSuccess ||
            hipMalloc(&sb.second, sizeof(double) * B) != hipSuccess)
            return fail(HELM_ENOMEM, "cnn: scale buffers");
    }
    hipLaunchKernelGGL(k_sample_scale<float>, dim3(B), dim3(256), 0, s, r, N, sqrtN, h2, sb.first, sb.second);
    HELM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pack<float>, dim3((unsigned)((N + 255) / 256), B), dim3(256), 0, s, r, N, sb.first, 1,
                       A->sol.t[A->sol.input].d, (float*)nullptr);
    HELM_CHECK_LAUNCH();
    if ((rc = run_forward(net, *A, A->sol, nullptr, 0, s))) return rc;
    // target and loss
    const long nout = (long)B * N * 2;
    static std::map<long, std::pair<float*, double*>> tbuf;
    auto& tb = tbuf[nout];
    const int nblk = (int)((nout + 255) / 256);
    if (!tb.first) {
        if (hipMalloc(&tb.first, sizeof(float) * nout) != hipSuccess ||
            hipMalloc(&tb.second, sizeof(double) * nblk) != hipSuccess)
            return fail(HELM_ENOMEM, "cnn: target buffers");
    }
    hipLaunchKernelGGL(k_target, dim3((unsigned)((N + 255) / 256), B), dim3(256), 0, s, e, N, sb.first, 1.0 / h2,
                       tb.first);
    HELM_CHECK_LAUNCH();
    Tens& yo = A->sol.t[A->sol.output];
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, A->sol.outf, tb.first, nout, 1.0f / B, yo.g, tb.second);
    HELM_CHECK_LAUNCH();
    if ((rc = run_backward(net, *A, A->sol, s))) return rc;
    for (int l = 0; l < 4; ++l) {
        Tens& z = A->enc.t[A->enc.z[l]];
        hipLaunchKernelGGL(k_batch_sum, g1(z.n()), dim3(256), 0, s, A->zg[l], B, z.n(), z.g);
        HELM_CHECK_LAUNCH();
    }
    if ((rc = run_backward(net, *A, A->enc, s))) return rc;
    if (loss) {
        std::vector<double> hp(nblk);
        HELM_HIP(hipMemcpyAsync(hp.data(), tb.second, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
        HELM_HIP(hipStreamSynchronize(s));
        double L = 0;
        for (double v : hp) L += v;
        *loss = L / B;
    }
    return HELM_OK;
}

static int adam_step(cnn_net* net, double lr, hipStream_t s) {
    net->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - std::pow(b1, (float)net->adam_t), c2 = 1.f - std::pow(b2, (float)net->adam_t);
    hipLaunchKernelGGL(k_adam, g1(net->nparam), dim3(256), 0, s, net->master, net->grad, net->adam_m, net->adam_v,
                       net->nparam, (float)lr, b1, b2, 1e-8f, c1, c2);
    HELM_CHECK_LAUNCH();
    return refresh_weights(net, s);
}

// (r, e) pairs of eq. (4.3) for samples first .. first+n-1 into R, E (c64).
static int make_pairs(const helm_op* op, int first, int n, uint32_t seed, c64* R, c64* E, hipStream_t s) {
    const long N = op->n();
    const long tot = (long)n * N;
    c128 *x, *xt, *ed;
    c64* b;
    if (hipMalloc(&x, sizeof(c128) * tot) != hipSuccess || hipMalloc(&xt, sizeof(c128) * tot) != hipSuccess ||
        hipMalloc(&ed, sizeof(c128) * tot) != hipSuccess || hipMalloc(&b, sizeof(c64) * tot) != hipSuccess)
        return fail(HELM_ENOMEM, "cnn: data generation buffers");
    int rc = HELM_OK;
    std::vector<int> ks(n);
    for (int i = 0; i < n; ++i) {
        u32x4 w = philox_at((uint64_t)(first + i), 0x7FFFFFFFu, seed, 0xDA7Au);
        ks[i] = 1 + (int)std::floor(10.0 * philox_u01(w.v[0]));
    }
    hipLaunchKernelGGL(k_randn_c, dim3((unsigned)((N + 255) / 256), n), dim3(256), 0, s, x, N, first, seed);
    if (hipGetLastError() != hipSuccess) rc = fail(HELM_EHIP, "cnn: randn launch");
    // b = H x (c128), cast to c64
    if (!rc) rc = launch_matvec<double>(op, x, ed, n, 0, s);
    if (!rc) hipLaunchKernelGGL(k_c128_to_c64, g1(tot), dim3(256), 0, s, ed, b, tot);
    // x~ = GMRES(H, M = V-cycle, b, x0 = 0, k iterations)
    if (!rc) rc = solve_fixed_iters(op, b, xt, n, ks.data(), 0, s);
    // e = x - x~, r = H e
    if (!rc) hipLaunchKernelGGL(k_sub_c128, g1(tot), dim3(256), 0, s, x, xt, ed, tot);
    if (!rc) rc = launch_matvec<double>(op, ed, x, n, 0, s);
    if (!rc) hipLaunchKernelGGL(k_c128_to_c64, g1(tot), dim3(256), 0, s, ed, E, tot);
    if (!rc) hipLaunchKernelGGL(k_c128_to_c64, g1(tot), dim3(256), 0, s, x, R, tot);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(HELM_EHIP, "cnn: data generation");
    (void)hipFree(x);
    (void)hipFree(xt);
    (void)hipFree(ed);
    (void)hipFree(b);
    return rc;
}

// Alg. 2 data epoch: for each (r, e) in R[0..n): e_new = M_net(r); e~ = one
// GMRES step (V-cycle) from e_new on H e = r; r~ = H e~  -> R[n..2n), E[n..2n).
static int alg2_epoch(cnn_net* net, const helm_op* op, c64* R, c64* E, int n, int chunk, hipStream_t s) {
    const long N = op->n();
    c128 *xe, *rr;
    c64* en;
    long tot = (long)chunk * N;
    if (hipMalloc(&xe, sizeof(c128) * tot) != hipSuccess || hipMalloc(&rr, sizeof(c128) * tot) != hipSuccess ||
        hipMalloc(&en, sizeof(c64) * tot) != hipSuccess)
        return fail(HELM_ENOMEM, "cnn: retraining buffers");
    int rc = HELM_OK;
    std::vector<int> ones(chunk, 1);
    for (int i0 = 0; i0 < n && !rc; i0 += chunk) {
        int nb = std::min(chunk, n - i0);
        long t = (long)nb * N;
        rc = apply_impl<float>(net, op, R + (long)i0 * N, nullptr, 0, en, nb, nullptr, 0, s);
        if (!rc) hipLaunchKernelGGL(k_c64_to_c128, g1(t), dim3(256), 0, s, en, xe, t);
        if (!rc) rc = solve_fixed_iters(op, R + (long)i0 * N, xe, nb, ones.data(), 1, s);
        if (!rc) rc = launch_matvec<double>(op, xe, rr, nb, 0, s);
        if (!rc) hipLaunchKernelGGL(k_c128_to_c64, g1(t), dim3(256), 0, s, xe, E + (long)(n + i0) * N, t);
        if (!rc) hipLaunchKernelGGL(k_c128_to_c64, g1(t), dim3(256), 0, s, rr, R + (long)(n + i0) * N, t);
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(HELM_EHIP, "cnn: retraining epoch");
    (void)hipFree(xe);
    (void)hipFree(rr);
    (void)hipFree(en);
    return rc;
}

}  // namespace helm

// ------------------------------------------------------------------ single-layer hooks
namespace helm {
namespace {
template <typename T>
T* dev_copy(const T* h, size_t n, std::vector<void*>& keep) {
    T* d = nullptr;
    if (hipMalloc(&d, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return nullptr;
    keep.push_back(d);
    if (h && hipMemcpy(d, h, sizeof(T) * n, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    if (!h && hipMemset(d, 0, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return nullptr;
    return d;
}
bf16* dev_bf16(const float* h, size_t n, std::vector<void*>& keep) {
    float* f = dev_copy(h, n, keep);
    bf16* b = dev_copy<bf16>(nullptr, n, keep);
    if (!f || !b) return nullptr;
    hipLaunchKernelGGL(k_f32_to_bf16, g1((long)n), dim3(256), 0, nullptr, f, b, (long)n);
    return b;
}
struct Keep {
    std::vector<void*> p;
    ~Keep() {
        (void)hipDeviceSynchronize();
        for (void* q : p) (void)hipFree(q);
    }
};
}  // namespace
}  // namespace helm

// ------------------------------------------------------------------ C ABI
extern "C" {

int cnn_create(const cnn_arch* arch, uint64_t seed, cnn_net_t* out) {
    if (!out) return fail(HELM_EINVAL, "cnn_create: out is NULL");
    *out = nullptr;
    cnn_net* n = new cnn_net();
    static std::atomic<uint64_t> next_uid{1};
    n->uid = next_uid++;
    if (arch) {
        for (int l = 0; l < 4; ++l)
            if (arch->widths[l] > 0) n->widths[l] = arch->widths[l];
        if (arch->down_res > 0) n->down_res = arch->down_res;
        for (int l = 0; l < 4; ++l)
            if (n->widths[l] % 32) {
                delete n;
                return fail(HELM_EINVAL, "cnn_create: widths must be multiples of 32");
            }
    }
    n->seed = seed;
    build_layers(n);
    if (hipMalloc(&n->master, sizeof(float) * n->nparam) != hipSuccess ||
        hipMalloc(&n->grad, sizeof(float) * n->nparam) != hipSuccess ||
        hipMalloc(&n->adam_m, sizeof(float) * n->nparam) != hipSuccess ||
        hipMalloc(&n->adam_v, sizeof(float) * n->nparam) != hipSuccess ||
        hipMalloc(&n->wb, sizeof(bf16) * n->nwb) != hipSuccess) {
        cnn_destroy(n);
        return fail(HELM_ENOMEM, "cnn_create: parameter allocation failed");
    }
    // He-normal weights from Philox (counter (index, layer), key (seed lo, seed hi)),
    // zero biases; the second convolution of every residual block starts at 0.1x
    // and the output layer at 0.01x, so that an untrained solver is close to
    // the zero map and M_VU starts close to the plain V-cycle.
    std::vector<float> h(n->nparam, 0.f);
    std::vector<double> gain(n->layers.size(), 1.0);
    gain.back() = 0.01;
    for (size_t li = 0; li + 1 < n->layers.size(); ++li) {
        const LayerDesc& L = n->layers[li];
        const LayerDesc& P = li > 0 ? n->layers[li - 1] : L;
        // a residual block is a pair of C -> C stride-1 convolutions
        if (li > 0 && L.kind == L_CONV && P.kind == L_CONV && L.cin == L.cout && P.cin == P.cout &&
            L.stride == 1 && P.stride == 1 && L.cin == P.cin && gain[li - 1] == 1.0)
            gain[li] = 0.1;
    }
    for (size_t li = 0; li < n->layers.size(); ++li) {
        const LayerDesc& L = n->layers[li];
        double sd = gain[li] * std::sqrt(2.0 / ((L.kind == L_CONV ? 9.0 : 1.0) * L.cin));
        for (long i = 0; i < L.nw; ++i) {
            u32x4 w = philox_at((uint64_t)i, (uint32_t)li, (uint32_t)seed, (uint32_t)(seed >> 32));
            double u0 = philox_u01(w.v[0]), u1 = philox_u01(w.v[1]);
            h[L.woff + i] = (float)(sd * std::sqrt(-2.0 * std::log(u0)) * std::cos(2.0 * M_PI * u1));
        }
    }
    if (hipMemcpy(n->master, h.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->grad, 0, sizeof(float) * n->nparam) != hipSuccess ||
        hipMemset(n->adam_m, 0, sizeof(float) * n->nparam) != hipSuccess ||
        hipMemset(n->adam_v, 0, sizeof(float) * n->nparam) != hipSuccess) {
        cnn_destroy(n);
        return fail(HELM_EHIP, "cnn_create: parameter upload failed");
    }
    int rc = refresh_weights(n, nullptr);
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(HELM_EHIP, "cnn_create: sync failed");
    if (rc) {
        cnn_destroy(n);
        return rc;
    }
    *out = n;
    return HELM_OK;
}

void cnn_destroy(cnn_net_t n) {
    if (!n) return;
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    (void)hipDeviceSynchronize();
    auto it = g_state.find(n);
    if (it != g_state.end()) {
        for (auto& kv : it->second.arenas) delete kv.second;
        g_state.erase(it);
    }
    if (n->master) (void)hipFree(n->master);
    if (n->grad) (void)hipFree(n->grad);
    if (n->adam_m) (void)hipFree(n->adam_m);
    if (n->adam_v) (void)hipFree(n->adam_v);
    if (n->wb) (void)hipFree(n->wb);
    delete n;
}

int cnn_num_params(cnn_net_t n, long* count) {
    if (!n || !count) return fail(HELM_EINVAL, "cnn_num_params: bad arguments");
    *count = n->nparam;
    return HELM_OK;
}

int cnn_get_params(cnn_net_t n, float* host) {
    if (!n || !host) return fail(HELM_EINVAL, "cnn_get_params: bad arguments");
    HELM_HIP(hipDeviceSynchronize());
    HELM_HIP(hipMemcpy(host, n->master, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    return HELM_OK;
}

int cnn_set_params(cnn_net_t n, const float* host) {
    if (!n || !host) return fail(HELM_EINVAL, "cnn_set_params: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    HELM_HIP(hipDeviceSynchronize());
    HELM_HIP(hipMemcpy(n->master, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    int rc = refresh_weights(n, nullptr);
    if (!rc) HELM_HIP(hipDeviceSynchronize());
    return rc;
}

int cnn_get_grad(cnn_net_t n, float* host) {
    if (!n || !host) return fail(HELM_EINVAL, "cnn_get_grad: bad arguments");
    HELM_HIP(hipDeviceSynchronize());
    HELM_HIP(hipMemcpy(host, n->grad, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    return HELM_OK;
}

int cnn_zero_grad(cnn_net_t n) {
    if (!n) return fail(HELM_EINVAL, "cnn_zero_grad: NULL net");
    HELM_HIP(hipMemset(n->grad, 0, sizeof(float) * n->nparam));
    return HELM_OK;
}

int cnn_save(cnn_net_t n, const char* path) {
    if (!n || !path) return fail(HELM_EINVAL, "cnn_save: bad arguments");
    std::vector<float> w(n->nparam), m(n->nparam), v(n->nparam);
    HELM_HIP(hipDeviceSynchronize());
    HELM_HIP(hipMemcpy(w.data(), n->master, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    HELM_HIP(hipMemcpy(m.data(), n->adam_m, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    HELM_HIP(hipMemcpy(v.data(), n->adam_v, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    FILE* f = fopen(path, "wb");
    if (!f) return fail(HELM_EINVAL, "cnn_save: cannot open %s", path);
    const char magic[8] = {'H', 'E', 'L', 'M', 'C', 'N', 'N', '1'};
    long hdr[8] = {n->widths[0], n->widths[1], n->widths[2], n->widths[3], n->down_res, n->nparam, n->adam_t,
                   (long)n->seed};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(hdr, sizeof(long), 8, f) == 8 &&
              fwrite(w.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam &&
              fwrite(m.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam &&
              fwrite(v.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam;
    fclose(f);
    return ok ? HELM_OK : fail(HELM_EINVAL, "cnn_save: write failed");
}

int cnn_load(const char* path, cnn_net_t* out) {
    if (!path || !out) return fail(HELM_EINVAL, "cnn_load: bad arguments");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(HELM_EINVAL, "cnn_load: cannot open %s", path);
    char magic[8];
    long hdr[8];
    if (fread(magic, 1, 8, f) != 8 || memcmp(magic, "HELMCNN1", 8) != 0 || fread(hdr, sizeof(long), 8, f) != 8) {
        fclose(f);
        return fail(HELM_EINVAL, "cnn_load: %s is not a network file", path);
    }
    cnn_arch arch{};
    for (int l = 0; l < 4; ++l) arch.widths[l] = (int)hdr[l];
    arch.down_res = (int)hdr[4];
    cnn_net_t n;
    int rc = cnn_create(&arch, (uint64_t)hdr[7], &n);
    if (rc) {
        fclose(f);
        return rc;
    }
    if (n->nparam != hdr[5]) {
        fclose(f);
        cnn_destroy(n);
        return fail(HELM_EINVAL, "cnn_load: parameter count mismatch");
    }
    std::vector<float> w(n->nparam), m(n->nparam), v(n->nparam);
    bool ok = fread(w.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam &&
              fread(m.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam &&
              fread(v.data(), sizeof(float), n->nparam, f) == (size_t)n->nparam;
    fclose(f);
    if (!ok) {
        cnn_destroy(n);
        return fail(HELM_EINVAL, "cnn_load: truncated file");
    }
    n->adam_t = hdr[6];
    if (hipMemcpy(n->adam_m, m.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->adam_v, v.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        (rc = cnn_set_params(n, w.data()))) {
        cnn_destroy(n);
        return rc ? rc : fail(HELM_EHIP, "cnn_load: upload failed");
    }
    *out = n;
    return HELM_OK;
}

int cnn_forward(cnn_net_t n, helm_op_t op, const float* rin, float* out, int B, void* stream) {
    if (!n || !op || !rin || !out || B <= 0) return fail(HELM_EINVAL, "cnn_forward: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = check_grid(op))) return rc;
    Arena* A;
    if ((rc = get_arena(n, B, op->nz, op->nx, false, &A))) return rc;
    if ((rc = ensure_encoded(n, op, A, s))) return rc;
    long ne = (long)B * op->n() * 2;
    hipLaunchKernelGGL(k_f32_to_bf16, g1(ne), dim3(256), 0, s, rin, A->sol.t[A->sol.input].d, ne);
    HELM_CHECK_LAUNCH();
    if ((rc = run_forward(n, *A, A->sol, nullptr, 0, s))) return rc;
    HELM_HIP(hipMemcpyAsync(out, A->sol.outf, sizeof(float) * ne, hipMemcpyDeviceToDevice, s));
    HELM_HIP(hipStreamSynchronize(s));
    return HELM_OK;
}


int cnn_layer_resblock(int B, int H, int W, const float* x, const float* w1, const float* b1, const float* w2,
                       const float* b2, float* out) {
    if (B <= 0 || H <= 0 || W <= 0 || !x || !w1 || !b1 || !w2 || !b2 || !out)
        return fail(HELM_EINVAL, "cnn_layer_resblock: bad arguments");
    Keep k;
    const long nw = 32L * 9 * 32, nx = (long)B * H * W * 32;
    const int K = pad32(9 * 32), Kt = pad32(9 * 32);
    float* w1d = dev_copy(w1, nw, k.p);
    float* w2d = dev_copy(w2, nw, k.p);
    float* b1d = dev_copy(b1, 32, k.p);
    float* b2d = dev_copy(b2, 32, k.p);
    bf16* f1 = dev_copy<bf16>(nullptr, 32L * K, k.p);
    bf16* f2 = dev_copy<bf16>(nullptr, 32L * K, k.p);
    bf16* t1 = dev_copy<bf16>(nullptr, 32L * Kt, k.p);
    bf16* t2 = dev_copy<bf16>(nullptr, 32L * Kt, k.p);
    bf16* xd = dev_bf16(x, nx, k.p);
    bf16* yd = dev_copy<bf16>(nullptr, nx, k.p);
    if (!w1d || !w2d || !b1d || !b2d || !f1 || !f2 || !t1 || !t2 || !xd || !yd) return fail(HELM_ENOMEM, "buffers");
    hipLaunchKernelGGL(k_refresh_conv, g1(32L * K), dim3(256), 0, nullptr, w1d, 32, 32, K, Kt, f1, t1);
    hipLaunchKernelGGL(k_refresh_conv, g1(32L * K), dim3(256), 0, nullptr, w2d, 32, 32, K, Kt, f2, t2);
    ResArgs r{};
    r.x = xd;
    r.B = B;
    r.H = H;
    r.W = W;
    r.w1 = f1;
    r.K1 = K;
    r.b1 = b1d;
    r.w2 = f2;
    r.K2 = K;
    r.b2 = b2d;
    r.out = yd;
    int rc = launch_resblock32(r, nullptr);
    if (rc) return rc;
    std::vector<bf16> hb(nx);
    HELM_HIP(hipMemcpy(hb.data(), yd, sizeof(bf16) * nx, hipMemcpyDeviceToHost));
    for (long i = 0; i < nx; ++i) out[i] = (float)hb[i];
    return HELM_OK;
}

int cnn_layer_forward(int kind, int stride, int B, int H, int W, int c1, int c2, int bcast2, int cout,
                      const float* x1, const float* x2, const float* w, const float* b, const float* resid, int relu,
                      float* out) {
    if (B <= 0 || H <= 0 || W <= 0 || c1 <= 0 || cout <= 0 || !x1 || !w || !b || !out || (kind != 0 && kind != 1))
        return fail(HELM_EINVAL, "cnn_layer_forward: bad arguments");
    if (kind == 1 && c2) return fail(HELM_EINVAL, "cnn_layer_forward: up-conv takes one source");
    Keep k;
    const int cin = c1 + c2;
    LayerDesc L{};
    L.kind = kind;
    L.cin = cin;
    L.cout = cout;
    L.K = kind == 0 ? pad32(9 * cin) : cin;
    L.Kt = kind == 0 ? pad32(9 * cout) : 4 * cout;
    long nw = kind == 0 ? (long)cout * 9 * cin : 4L * cout * cin;
    float* wd = dev_copy(w, nw, k.p);
    float* bd = dev_copy(b, cout, k.p);
    long nwf = kind == 0 ? (long)cout * L.K : 4L * cout * cin;
    long nwt = (long)cin * L.Kt;
    bf16* wf = dev_copy<bf16>(nullptr, nwf, k.p);
    bf16* wt = dev_copy<bf16>(nullptr, nwt, k.p);
    const int Ho = kind == 0 ? (H + stride - 1) / stride : 2 * H, Wo = kind == 0 ? (W + stride - 1) / stride : 2 * W;
    long nx1 = (long)B * H * W * c1, nx2 = (long)(bcast2 ? 1 : B) * H * W * c2, ny = (long)B * Ho * Wo * cout;
    bf16* x1d = dev_bf16(x1, nx1, k.p);
    bf16* x2d = c2 ? dev_bf16(x2, nx2, k.p) : nullptr;
    bf16* rd = resid ? dev_bf16(resid, ny, k.p) : nullptr;
    bf16* yd = dev_copy<bf16>(nullptr, ny, k.p);
    float* yf = dev_copy<float>(nullptr, ny, k.p);
    if (!wd || !bd || !wf || !wt || !x1d || (c2 && !x2d) || !yd || !yf) return fail(HELM_ENOMEM, "layer buffers");
    if (kind == 0)
        hipLaunchKernelGGL(k_refresh_conv, g1(std::max(nwf, nwt)), dim3(256), 0, nullptr, wd, cout, cin, L.K, L.Kt, wf,
                           wt);
    else
        hipLaunchKernelGGL(k_refresh_up, g1(nw), dim3(256), 0, nullptr, wd, cout, cin, wf, wt);
    GemmArgs g{};
    g.a1 = x1d;
    g.c1 = c1;
    g.abs1 = (long)H * W * c1;
    g.a2 = x2d;
    g.c2 = c2;
    g.abs2 = bcast2 ? 0 : (long)H * W * c2;
    g.B = B;
    g.Hi = H;
    g.Wi = W;
    g.stride = stride;
    g.w = wf;
    g.K = L.K;
    g.bias = bd;
    g.relu = relu;
    g.out = yd;
    if (kind == 0) {
        g.gmode = G_CONV;
        g.Ho = Ho;
        g.Wo = Wo;
        g.N = cout;
        g.kvalid = 9 * cin;
        g.epi = E_FWD;
        g.resid = rd;
        g.outf = yf;
        g.M = (long)B * Ho * Wo;
    } else {
        g.gmode = G_UP;
        g.Ho = H;
        g.Wo = W;
        g.N = 4 * cout;
        g.kvalid = cin;
        g.epi = E_UPFWD;
        g.M = (long)B * H * W;
    }
    int rc = launch_gemm(g, nullptr);
    if (rc) return rc;
    if (kind == 1) {
        // up-conv writes bf16 only
        std::vector<bf16> hb(ny);
        HELM_HIP(hipMemcpy(hb.data(), yd, sizeof(bf16) * ny, hipMemcpyDeviceToHost));
        for (long i = 0; i < ny; ++i) out[i] = (float)hb[i];
        return HELM_OK;
    }
    HELM_HIP(hipMemcpy(out, yf, sizeof(float) * ny, hipMemcpyDeviceToHost));
    return HELM_OK;
}

int cnn_layer_backward(int kind, int stride, int B, int H, int W, int c1, int c2, int bcast2, int cout,
                       const float* x1, const float* x2, const float* w, const float* y, int relu, const float* gout,
                       float* gx1, float* gx2, float* gw, float* gb) {
    if (B <= 0 || H <= 0 || W <= 0 || c1 <= 0 || cout <= 0 || !x1 || !w || !y || !gout || !gx1 || !gw || !gb ||
        (kind != 0 && kind != 1) || (c2 && !gx2))
        return fail(HELM_EINVAL, "cnn_layer_backward: bad arguments");
    Keep k;
    const int cin = c1 + c2;
    const int K = kind == 0 ? pad32(9 * cin) : cin;
    const int Kt = kind == 0 ? pad32(9 * cout) : 4 * cout;
    long nw = kind == 0 ? (long)cout * 9 * cin : 4L * cout * cin;
    long nwf = kind == 0 ? (long)cout * K : nw, nwt = (long)cin * Kt;
    const int Ho = kind == 0 ? (H + stride - 1) / stride : 2 * H, Wo = kind == 0 ? (W + stride - 1) / stride : 2 * W;
    long nx1 = (long)B * H * W * c1, nx2b = (long)B * H * W * c2, nx2 = (long)(bcast2 ? 1 : B) * H * W * c2;
    long ny = (long)B * Ho * Wo * cout;
    float* wd = dev_copy(w, nw, k.p);
    bf16* wf = dev_copy<bf16>(nullptr, nwf, k.p);
    bf16* wt = dev_copy<bf16>(nullptr, nwt, k.p);
    bf16* x1d = dev_bf16(x1, nx1, k.p);
    bf16* x2d = c2 ? dev_bf16(x2, nx2, k.p) : nullptr;
    bf16* yd = dev_bf16(y, ny, k.p);
    float* gd = dev_copy(gout, ny, k.p);
    bf16* gm = dev_copy<bf16>(nullptr, ny, k.p);
    float* g1d = dev_copy<float>(nullptr, nx1, k.p);
    float* g2d = c2 ? dev_copy<float>(nullptr, nx2b, k.p) : nullptr;
    float* gwd = dev_copy<float>(nullptr, nw, k.p);
    long P = kind == 0 ? (long)B * Ho * Wo : (long)B * H * W;
    int M = kind == 0 ? cout : 4 * cout, N = kind == 0 ? 9 * cin : cin, Npad = (N + 63) / 64 * 64;
    int nsplit = 8;
    const size_t nbias = (size_t)((ny + BIAS_STEPS * 8 - 1) / (BIAS_STEPS * 8)) * cout;
    float* part = dev_copy<float>(nullptr, (size_t)nsplit * M * Npad + nbias, k.p);
    if (!wd || !wf || !wt || !x1d || !yd || !gd || !gm || !g1d || !gwd || !part) return fail(HELM_ENOMEM, "buffers");
    if (kind == 0)
        hipLaunchKernelGGL(k_refresh_conv, g1(std::max(nwf, nwt)), dim3(256), 0, nullptr, wd, cout, cin, K, Kt, wf, wt);
    else
        hipLaunchKernelGGL(k_refresh_up, g1(nw), dim3(256), 0, nullptr, wd, cout, cin, wf, wt);
    hipLaunchKernelGGL(k_relu_bwd, g1(ny), dim3(256), 0, nullptr, gd, yd, ny, relu, gm);
    // bias (reduction over the output pixels)
    float* bpart = part + (size_t)nsplit * M * Npad;
    float* gbd = dev_copy<float>(nullptr, cout, k.p);
    if (!gbd) return fail(HELM_ENOMEM, "buffers");
    int rc = bias_grad(gm, ny, cout, bpart, nbias, gbd, nullptr);
    if (rc) return rc;
    // weights
    WgradArgs wa{};
    wa.g = gm;
    wa.Hg = Ho;
    wa.Wg = Wo;
    wa.Cg = cout;
    wa.a1 = x1d;
    wa.c1 = c1;
    wa.abs1 = (long)H * W * c1;
    wa.a2 = x2d;
    wa.c2 = c2;
    wa.abs2 = bcast2 ? 0 : (long)H * W * c2;
    wa.B = B;
    wa.Hi = H;
    wa.Wi = W;
    wa.stride = stride;
    wa.mode = kind == 0 ? G_CONV : G_UP;
    wa.M = M;
    wa.N = N;
    wa.Npad = Npad;
    wa.P = P;
    wa.part = part;
    rc = launch_wgrad(wa, nsplit, nullptr, &nsplit);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_wsplits, g1(nw), dim3(256), 0, nullptr, part, nsplit, M, N, Npad, gwd);
    // data
    GemmArgs g{};
    g.a1 = gm;
    g.c1 = cout;
    g.abs1 = (long)Ho * Wo * cout;
    g.B = B;
    g.Hi = Ho;
    g.Wi = Wo;
    g.stride = stride;
    g.w = wt;
    g.K = Kt;
    g.epi = E_ACC;
    g.Ho = H;
    g.Wo = W;
    g.M = (long)B * H * W;
    g.acc1 = g1d;
    g.acc2 = g2d;
    g.n1 = c1;
    g.N = cin;
    g.gmode = kind == 0 ? G_CONVT : G_UPT;
    g.kvalid = kind == 0 ? 9 * cout : 4 * cout;
    if ((rc = launch_gemm(g, nullptr))) return rc;
    HELM_HIP(hipMemcpy(gx1, g1d, sizeof(float) * nx1, hipMemcpyDeviceToHost));
    if (c2) HELM_HIP(hipMemcpy(gx2, g2d, sizeof(float) * nx2b, hipMemcpyDeviceToHost));
    HELM_HIP(hipMemcpy(gw, gwd, sizeof(float) * nw, hipMemcpyDeviceToHost));
    HELM_HIP(hipMemcpy(gb, gbd, sizeof(float) * cout, hipMemcpyDeviceToHost));
    return HELM_OK;
}

int cnn_precond_apply(cnn_net_t n, helm_op_t op, const void* r, void* e, int nrhs, void* stream) {
    if (!n || !op || nrhs < 0) return fail(HELM_EINVAL, "cnn_precond_apply: bad arguments");
    if (nrhs == 0) return HELM_OK;   // an empty batch: the buffers may be NULL
    if (!r || !e) return fail(HELM_EINVAL, "cnn_precond_apply: NULL buffer");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    return apply_impl<float>(n, op, (const c64*)r, nullptr, 0, (c64*)e, nrhs, nullptr, 0, (hipStream_t)stream);
}

int cnn_loss_grad(cnn_net_t n, helm_op_t op, const void* r, const void* e, int B, double* loss, void* stream) {
    if (!n || !op || !r || !e || B <= 0) return fail(HELM_EINVAL, "cnn_loss_grad: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    return loss_grad(n, op, (const c64*)r, (const c64*)e, B, loss, (hipStream_t)stream);
}

int cnn_adam_step(cnn_net_t n, double lr, void* stream) {
    if (!n || !(lr > 0)) return fail(HELM_EINVAL, "cnn_adam_step: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    int rc = adam_step(n, lr, (hipStream_t)stream);
    if (!rc) HELM_HIP(hipStreamSynchronize((hipStream_t)stream));
    return rc;
}

int cnn_make_pairs(helm_op_t op, int first, int npairs, uint64_t seed, void* r, void* e, void* stream) {
    if (!op || !r || !e || npairs <= 0) return fail(HELM_EINVAL, "cnn_make_pairs: bad arguments");
    return make_pairs(op, first, npairs, (uint32_t)seed, (c64*)r, (c64*)e, (hipStream_t)stream);
}

int cnn_alg2_epoch(cnn_net_t n, helm_op_t op, void* r, void* e, int npairs, void* stream) {
    if (!n || !op || !r || !e || npairs <= 0) return fail(HELM_EINVAL, "cnn_alg2_epoch: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    return alg2_epoch(n, op, (c64*)r, (c64*)e, npairs, 32, (hipStream_t)stream);
}

int cnn_precond_train(cnn_net_t n, helm_op_t op, const cnn_train_opts* opt, uint64_t seed, float* loss_hist,
                      void* stream) {
    if (!n || !op || !opt) return fail(HELM_EINVAL, "cnn_precond_train: bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_cnn_mutex);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = check_grid(op))) return rc;
    const int B = opt->batch > 0 ? opt->batch : 16;
    const double lr = opt->lr > 0 ? opt->lr : 1e-4;
    const bool alg2 = opt->alg2_initial > 0;
    const int n0 = alg2 ? opt->alg2_initial : (opt->npairs > 0 ? opt->npairs : 2000);
    const int depochs = alg2 ? std::max(0, opt->alg2_data_epochs) : 0;
    const long N = op->n();
    const long cap = (long)n0 << depochs;
    c64 *R, *E;
    if (hipMalloc(&R, sizeof(c64) * cap * N) != hipSuccess || hipMalloc(&E, sizeof(c64) * cap * N) != hipSuccess)
        return fail(HELM_ENOMEM, "cnn_precond_train: dataset of %ld pairs", cap);
    c64 *rb, *eb;
    if (hipMalloc(&rb, sizeof(c64) * B * N) != hipSuccess || hipMalloc(&eb, sizeof(c64) * B * N) != hipSuccess) {
        (void)hipFree(R);
        (void)hipFree(E);
        return fail(HELM_ENOMEM, "cnn_precond_train: batch buffers");
    }
    // generate in chunks of 64 samples
    for (int i0 = 0; i0 < n0 && !rc; i0 += 64) {
        int nb = std::min(64, n0 - i0);
        rc = make_pairs(op, i0, nb, (uint32_t)seed, R + (long)i0 * N, E + (long)i0 * N, s);
    }
    long dsize = n0;
    long step = 0;
    const long total_steps = opt->steps > 0 ? opt->steps : 200;
    const int epochs = alg2 ? std::max(1, opt->alg2_epochs) : 1 << 30;
    for (int ep = 0; ep < epochs && step < total_steps && !rc; ++ep) {
        // one pass over D in a Philox permutation (sort by key)
        std::vector<std::pair<uint32_t, long>> perm(dsize);
        for (long i = 0; i < dsize; ++i)
            perm[i] = {philox_at((uint64_t)i, 0x5EEDu + ep, (uint32_t)seed, 0xA1B2u).v[0], i};
        std::sort(perm.begin(), perm.end());
        for (long b0 = 0; b0 + B <= dsize && step < total_steps && !rc; b0 += B) {
            for (int q = 0; q < B; ++q) {
                long i = perm[b0 + q].second;
                if (hipMemcpyAsync(rb + (long)q * N, R + i * N, sizeof(c64) * N, hipMemcpyDeviceToDevice, s) !=
                        hipSuccess ||
                    hipMemcpyAsync(eb + (long)q * N, E + i * N, sizeof(c64) * N, hipMemcpyDeviceToDevice, s) !=
                        hipSuccess)
                    rc = fail(HELM_EHIP, "cnn_precond_train: batch copy");
            }
            double L = 0;
            if (!rc) rc = loss_grad(n, op, rb, eb, B, loss_hist ? &L : nullptr, s);
            if (!rc) rc = adam_step(n, lr, s);
            if (!rc && loss_hist) loss_hist[step] = (float)L;
            ++step;
        }
        if (alg2 && ep < depochs && !rc) {
            rc = alg2_epoch(n, op, R, E, (int)dsize, 32, s);
            dsize *= 2;
        }
        if (!alg2 && dsize < B) break;
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(HELM_EHIP, "cnn_precond_train: sync");
    (void)hipFree(R);
    (void)hipFree(E);
    (void)hipFree(rb);
    (void)hipFree(eb);
    if (!rc && opt->steps_done) *opt->steps_done = (int)step;
    if (!rc && opt->dataset_size) *opt->dataset_size = (int)dsize;
    return rc;
}

}  // extern "C"

extern "C" int helm_autotune(int enable, int* tuned_shapes) {
    if (enable < -1 || enable > 2) return fail(HELM_EINVAL, "helm_autotune: enable must be -1, 0, 1 or 2");
    return conv_autotune(enable, tuned_shapes);
}

extern "C" int helm_conv_force(int kernel, int* kernel_count) { return conv_force(kernel, kernel_count); }

extern "C" int helm_autotune_file(const char* path, int save) {
    if (!path) return fail(HELM_EINVAL, "helm_autotune_file: path is NULL");
    return conv_autotune_file(path, save);
}
