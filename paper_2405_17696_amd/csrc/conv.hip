// Implicit-GEMM convolution kernels on the gfx950 BF16 matrix cores.
//
// One GEMM kernel serves the forward 3x3 convolutions (stride 1 or 2, one or
// two concatenated sources, fused bias / residual / ReLU), the 2x2 up-sampling
// convolutions, and both data gradients; a second kernel forms the weight
// gradients with the reduction over pixels split across workgroups.
//
// MFMA v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16] and D[4(l/16)+i][l%16], i = 0..3.
#include "conv.h"

namespace helm {

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Pixel (b, y, x) of row m of a B x Ho x Wo grid.
struct Pix {
    int b, y, x;
};
__device__ __forceinline__ Pix pix_of(long m, int Ho, int Wo) {
    Pix p;
    long hw = (long)Ho * Wo;
    p.b = (int)(m / hw);
    long r = m - (long)p.b * hw;
    p.y = (int)(r / Wo);
    p.x = (int)(r - (long)p.y * Wo);
    return p;
}

// 8 consecutive k's of row m starting at k0 (k0 % 8 == 0).
template <int GM>
__device__ __forceinline__ bf16x8 gather8(const GemmArgs& a, long m, int k0) {
    if (m >= a.M || k0 >= a.kvalid) return zero8();
    const Pix p = pix_of(m, a.Ho, a.Wo);
    const int C = a.c1 + a.c2;
    if (GM == G_CONV || GM == G_CONVT) {
        if ((C & 7) != 0 || k0 + 8 > a.kvalid) {
            // small-channel path (first layer): element by element
            bf16x8 v = zero8();
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int k = k0 + e;
                if (k >= a.kvalid) break;
                int tap = k / C, c = k - tap * C;
                int ky = tap / 3, kx = tap - ky * 3;
                int yi, xi;
                if (GM == G_CONV) {
                    yi = p.y * a.stride + ky - 1;
                    xi = p.x * a.stride + kx - 1;
                } else {
                    yi = p.y + 1 - ky;
                    xi = p.x + 1 - kx;
                    if (a.stride == 2) {
                        if ((yi | xi) & 1) continue;
                        yi >>= 1;
                        xi >>= 1;
                    }
                }
                if (yi < 0 || yi >= a.Hi || xi < 0 || xi >= a.Wi) continue;
                const bf16* src = c < a.c1 ? a.a1 + p.b * a.abs1 : a.a2 + p.b * a.abs2;
                int cc = c < a.c1 ? c : c - a.c1;
                int cs = c < a.c1 ? a.c1 : a.c2;
                v[e] = src[((long)yi * a.Wi + xi) * cs + cc];
            }
            return v;
        }
        int tap = k0 / C, c = k0 - tap * C;
        int ky = tap / 3, kx = tap - ky * 3;
        int yi, xi;
        if (GM == G_CONV) {
            yi = p.y * a.stride + ky - 1;
            xi = p.x * a.stride + kx - 1;
        } else {
            yi = p.y + 1 - ky;
            xi = p.x + 1 - kx;
            if (a.stride == 2) {
                if ((yi | xi) & 1) return zero8();
                yi >>= 1;
                xi >>= 1;
            }
        }
        if (yi < 0 || yi >= a.Hi || xi < 0 || xi >= a.Wi) return zero8();
        if (c < a.c1) return ld8(a.a1 + p.b * a.abs1 + ((long)yi * a.Wi + xi) * a.c1 + c);
        return ld8(a.a2 + p.b * a.abs2 + ((long)yi * a.Wi + xi) * a.c2 + (c - a.c1));
    } else if (GM == G_UP) {
        return ld8(a.a1 + p.b * a.abs1 + ((long)p.y * a.Wi + p.x) * a.c1 + k0);
    } else {  // G_UPT: k = (2a+d)*C + c, source (2y+a, 2x+d) of a 2Ho x 2Wo tensor
        int ad = k0 / a.c1, c = k0 - ad * a.c1;
        int yi = 2 * p.y + (ad >> 1), xi = 2 * p.x + (ad & 1);
        return ld8(a.a1 + p.b * a.abs1 + ((long)yi * a.Wi + xi) * a.c1 + c);
    }
}

constexpr int KC = 32;      // k per chunk
constexpr int LDS_K = 40;   // padded row length (bf16) of the LDS tiles

// D[M x N] = A[M x K] B^T  with B stored [N][K].  Block = 4 waves; block tile
// BM x BN with waves WGM x WGN, each wave (BM/WGM) x (BN/WGN) in 16x16 MFMA tiles.
template <int GM, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a, unsigned long long* wc) {
    constexpr int WTM = BM / WGM / 16;  // MFMA tiles per wave along M
    constexpr int WTN = BN / WGN / 16;
    constexpr int ASEG = BM * KC / 8;   // 16-byte segments per A chunk
    constexpr int BSEG = BN * KC / 8;
    constexpr int AS_PER_T = (ASEG + 255) / 256;
    constexpr int BS_PER_T = (BSEG + 255) / 256;
    __shared__ bf16 As[2][BM][LDS_K];
    __shared__ bf16 Bs[2][BN][LDS_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const long m0 = (long)blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    const int nchunk = a.K / KC;
    if (a.st && ((long)a.Ho * a.Wo) % BM == 0) {
        // a tile never straddles two samples when Ho*Wo is a multiple of BM
        const int b = (int)(m0 / ((long)a.Ho * a.Wo));
        const RhsState& S = a.st[a.rhs0 + b];
        if (!S.active || S.cycdone) return;
    }
    if (wc && tid == 0) {
        long mr = a.M - m0 < BM ? a.M - m0 : BM;
        int nr = a.N - n0 < BN ? a.N - n0 : BN;
        atomicAdd(wc, (unsigned long long)(2ull * mr * nr * (unsigned long long)a.kvalid));
    }

    bf16x8 ra[AS_PER_T], rb[BS_PER_T];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int q = 0; q < AS_PER_T; ++q) {
            int sgi = tid + q * 256;
            if (sgi < ASEG) {
                int row = sgi >> 2, sub = sgi & 3;
                ra[q] = gather8<GM>(a, m0 + row, kc * KC + sub * 8);
            }
        }
#pragma unroll
        for (int q = 0; q < BS_PER_T; ++q) {
            int sgi = tid + q * 256;
            if (sgi < BSEG) {
                int row = sgi >> 2, sub = sgi & 3;
                int n = n0 + row;
                rb[q] = n < a.N ? ld8(a.w + (long)n * a.K + kc * KC + sub * 8) : zero8();
            }
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AS_PER_T; ++q) {
            int sgi = tid + q * 256;
            if (sgi < ASEG) *reinterpret_cast<bf16x8*>(&As[buf][sgi >> 2][(sgi & 3) * 8]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BS_PER_T; ++q) {
            int sgi = tid + q * 256;
            if (sgi < BSEG) *reinterpret_cast<bf16x8*>(&Bs[buf][sgi >> 2][(sgi & 3) * 8]) = rb[q];
        }
    };

    f32x4 acc[WTM][WTN];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int kc = 0; kc < nchunk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nchunk) load_chunk(kc + 1);
        bf16x8 fa[WTM], fb[WTN];
#pragma unroll
        for (int i = 0; i < WTM; ++i)
            fa[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * (BM / WGM) + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int j = 0; j < WTN; ++j)
            fb[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * (BN / WGN) + j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
            for (int j = 0; j < WTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (kc + 1 < nchunk) {
            store_chunk(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int n = n0 + wn * (BN / WGN) + j * 16 + (lane & 15);
            if (n >= a.N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long m = m0 + wm * (BM / WGM) + i * 16 + (lane >> 4) * 4 + e;
                if (m >= a.M) continue;
                float v = acc[i][j][e];
                if (a.epi == E_FWD) {
                    v += a.bias[n];
                    if (a.resid) v += (float)a.resid[m * a.N + n];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    a.out[m * a.N + n] = (bf16)v;
                    if (a.outf) a.outf[m * a.N + n] = v;
                } else if (a.epi == E_UPFWD) {
                    const int cout = a.N >> 2;
                    const int ad = n / cout, co = n - ad * cout;
                    const Pix p = pix_of(m, a.Ho, a.Wo);
                    long o = (((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) * cout + co;
                    v += a.bias[co];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    a.out[o] = (bf16)v;
                } else {  // E_ACC
                    if (n < a.n1)
                        a.acc1[m * a.n1 + n] += v;
                    else
                        a.acc2[m * (a.N - a.n1) + (n - a.n1)] += v;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ halo-tiled 3x3 stride-1 convolution
// A block computes a 16 x 16 pixel tile of one sample for BN output channels.
// Per chunk of 32 input channels it stages the 18 x 18 input patch and the 9
// taps of the weights in LDS once and runs all nine taps from there (the
// implicit-GEMM kernel above re-reads every input pixel nine times through L2).
// FLIP = 1 runs the data gradient of a stride-1 convolution: taps mirrored,
// weights [Cin][tap][Cout].
constexpr int HT = 16;              // tile edge (pixels)
constexpr int HP = HT + 2;          // patch edge
constexpr int HC = 32;              // channels per chunk
constexpr int HLD = HC + 8;         // padded LDS row (bf16)

template <int BN, int FLIP, int EPI>
__global__ __launch_bounds__(256) void k_conv3_halo(GemmArgs a, unsigned long long* wc) {
    constexpr int WTN = BN / 16;    // MFMA tiles per wave along N
    __shared__ bf16 Ps[HP * HP][HLD];
    __shared__ bf16 Ws[9][BN][HLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (a.Wo + HT - 1) / HT, tiles_y = (a.Ho + HT - 1) / HT;
    int t = blockIdx.x;
    const int tx0 = (t % tiles_x) * HT;
    t /= tiles_x;
    const int ty0 = (t % tiles_y) * HT;
    const int b = t / tiles_y;
    const int n0 = blockIdx.y * BN;
    if (a.st && !(a.st[a.rhs0 + b].active && !a.st[a.rhs0 + b].cycdone)) return;
    const int C = a.c1 + a.c2;
    if (wc && tid == 0) {
        int my = a.Ho - ty0 < HT ? a.Ho - ty0 : HT, mx = a.Wo - tx0 < HT ? a.Wo - tx0 : HT;
        int nr = a.N - n0 < BN ? a.N - n0 : BN;
        atomicAdd(wc, 2ull * my * mx * nr * (unsigned long long)(9 * C));
    }
    f32x4 acc[4][WTN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    constexpr int PSEG = HP * HP * (HC / 8);        // 1296 16-byte segments of the patch
    constexpr int WSEG = 9 * BN * (HC / 8);         // weight segments
    constexpr int PPT = (PSEG + 255) / 256, WPT = (WSEG + 255) / 256;
    bf16x8 rp[PPT], rw[WPT];
    auto load = [&](int c0) {
        const bool s2 = c0 >= a.c1;
        const bf16* src = s2 ? a.a2 + b * a.abs2 : a.a1 + b * a.abs1;
        const int cs = s2 ? a.c2 : a.c1, cc = s2 ? c0 - a.c1 : c0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            int sg = tid + q * 256;
            if (sg >= PSEG) break;
            int pix = sg >> 2, sub = sg & 3;
            int py = pix / HP, px = pix - py * HP;
            int yi = ty0 + py - 1, xi = tx0 + px - 1;
            rp[q] = (yi >= 0 && yi < a.Hi && xi >= 0 && xi < a.Wi)
                        ? ld8(src + ((long)yi * a.Wi + xi) * cs + cc + sub * 8)
                        : zero8();
        }
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            int sg = tid + q * 256;
            if (sg >= WSEG) break;
            int row = sg >> 2, sub = sg & 3;        // row = tap * BN + n
            int tap = row / BN, n = row - tap * BN;
            rw[q] = n0 + n < a.N ? ld8(a.w + (long)(n0 + n) * a.K + tap * C + c0 + sub * 8) : zero8();
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            int sg = tid + q * 256;
            if (sg >= PSEG) break;
            *reinterpret_cast<bf16x8*>(&Ps[sg >> 2][(sg & 3) * 8]) = rp[q];
        }
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            int sg = tid + q * 256;
            if (sg >= WSEG) break;
            int row = sg >> 2;
            *reinterpret_cast<bf16x8*>(&Ws[row / BN][row % BN][(sg & 3) * 8]) = rw[q];
        }
    };
    const int nchunk = C / HC;
    load(0);
    for (int ch = 0; ch < nchunk; ++ch) {
        store();
        __syncthreads();
        if (ch + 1 < nchunk) load((ch + 1) * HC);
        // wave w: tile rows 4w .. 4w+3, each a 16-pixel MFMA row tile
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = FLIP ? 2 - tap / 3 : tap / 3, kx = FLIP ? 2 - tap % 3 : tap % 3;
            bf16x8 fb[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                fb[j] = *reinterpret_cast<const bf16x8*>(&Ws[tap][j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ty = wave * 4 + i;
                bf16x8 fa = *reinterpret_cast<const bf16x8*>(&Ps[(ty + ky) * HP + (lane & 15) + kx][(lane >> 4) * 8]);
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: acc[i][j][e] = D[pixel (ty = 4w+i, tx = 4(l/16)+e)][n = j*16 + l%16]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ty0 + wave * 4 + i;
        if (y >= a.Ho) continue;
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int n = n0 + j * 16 + (lane & 15);
            if (n >= a.N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = tx0 + (lane >> 4) * 4 + e;
                if (x >= a.Wo) continue;
                const long m = ((long)b * a.Ho + y) * a.Wo + x;
                float v = acc[i][j][e];
                if (EPI == E_FWD) {
                    v += a.bias[n];
                    if (a.resid) v += (float)a.resid[m * a.N + n];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    a.out[m * a.N + n] = (bf16)v;
                    if (a.outf) a.outf[m * a.N + n] = v;
                } else {
                    if (n < a.n1)
                        a.acc1[m * a.n1 + n] += v;
                    else
                        a.acc2[m * (a.N - a.n1) + (n - a.n1)] += v;
                }
            }
        }
    }
}

// The halo kernel applies when every source has a multiple of 32 channels.
static bool halo_ok(const GemmArgs& a) {
    if (!(a.gmode == G_CONV || a.gmode == G_CONVT) || a.stride != 1) return false;
    if (a.c1 % HC || a.c2 % HC) return false;
    if (a.gmode == G_CONV && a.epi != E_FWD) return false;
    if (a.gmode == G_CONVT && a.epi != E_ACC) return false;
    return a.K >= 9 * (a.c1 + a.c2);
}

static int launch_halo(const GemmArgs& a, hipStream_t s) {
    unsigned long long* wc = WORK_COUNTER("k_conv");
    const int tiles = ((a.Ho + HT - 1) / HT) * ((a.Wo + HT - 1) / HT) * a.B;
    const bool flip = a.gmode == G_CONVT;
    if (a.N <= 32) {
        dim3 grid(tiles, (a.N + 31) / 32);
        if (flip)
            TIMED_LAUNCH("k_conv", s, (k_conv3_halo<32, 1, E_ACC>), grid, dim3(256), 0, s, a, wc);
        else
            TIMED_LAUNCH("k_conv", s, (k_conv3_halo<32, 0, E_FWD>), grid, dim3(256), 0, s, a, wc);
    } else {
        dim3 grid(tiles, (a.N + 63) / 64);
        if (flip)
            TIMED_LAUNCH("k_conv", s, (k_conv3_halo<64, 1, E_ACC>), grid, dim3(256), 0, s, a, wc);
        else
            TIMED_LAUNCH("k_conv", s, (k_conv3_halo<64, 0, E_FWD>), grid, dim3(256), 0, s, a, wc);
    }
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

template <int GM>
static int launch_gemm_mode(const GemmArgs& a, hipStream_t s) {
    unsigned long long* wc = WORK_COUNTER("k_conv");
    if (a.N <= 32) {
        dim3 grid((unsigned)((a.M + 127) / 128), (a.N + 31) / 32);
        TIMED_LAUNCH("k_conv", s, (k_gemm<GM, 128, 32, 4, 1>), grid, dim3(256), 0, s, a, wc);
    } else {
        dim3 grid((unsigned)((a.M + 63) / 64), (a.N + 63) / 64);
        TIMED_LAUNCH("k_conv", s, (k_gemm<GM, 64, 64, 2, 2>), grid, dim3(256), 0, s, a, wc);
    }
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

int launch_gemm(const GemmArgs& a, hipStream_t s) {
    if (a.K % KC != 0) return fail(HELM_EINVAL, "gemm: K=%d not a multiple of %d", a.K, KC);
    if (a.M <= 0 || a.N <= 0) return HELM_OK;
    if (halo_ok(a)) return launch_halo(a, s);
    switch (a.gmode) {
        case G_CONV:
            return launch_gemm_mode<G_CONV>(a, s);
        case G_CONVT:
            return launch_gemm_mode<G_CONVT>(a, s);
        case G_UP:
            return launch_gemm_mode<G_UP>(a, s);
        case G_UPT:
            return launch_gemm_mode<G_UPT>(a, s);
        default:
            return fail(HELM_EINVAL, "gemm: gather mode %d", a.gmode);
    }
}

// ------------------------------------------------------------------ weight gradient
// dW[row][k] = sum over pixels p of g(row, p) * x(p, k), split over pixel chunks.
// LDS holds both operands transposed ([row][pixel], [k][pixel]) so that the
// MFMA fragments are 16-byte reads.
constexpr int WG_BM = 32, WG_BN = 64, WG_KP = 32;

__device__ __forceinline__ bf16x8 wg_gather_x(const WgradArgs& a, long pix, int k0) {
    // x(p, k0..k0+7) of the forward A operand; p indexes the forward row grid
    if (pix >= a.P) return zero8();
    GemmArgs g{};
    g.a1 = a.a1;
    g.a2 = a.a2;
    g.c1 = a.c1;
    g.c2 = a.c2;
    g.abs1 = a.abs1;
    g.abs2 = a.abs2;
    g.B = a.B;
    g.Hi = a.Hi;
    g.Wi = a.Wi;
    g.stride = a.stride;
    g.M = a.P;
    if (a.mode == G_CONV) {
        g.Ho = a.Hg;
        g.Wo = a.Wg;
        g.kvalid = 9 * (a.c1 + a.c2);
        return gather8<G_CONV>(g, pix, k0);
    }
    g.Ho = a.Hi;
    g.Wo = a.Wi;
    g.kvalid = a.c1;
    if (k0 >= a.c1) return zero8();
    return gather8<G_UP>(g, pix, k0);
}

__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
    __shared__ bf16 Ag[WG_BM][WG_KP + 8];
    __shared__ bf16 Bx[WG_BN][WG_KP + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.y * WG_BM, c0 = blockIdx.x * WG_BN;
    const long p_begin = (long)blockIdx.z * a.pchunk;
    const long p_end = p_begin + a.pchunk < a.P ? p_begin + a.pchunk : a.P;
    // wave w: rows 0..31 (two 16-row tiles), columns w*16 .. w*16+15
    f32x4 acc[2] = {(f32x4){0.f, 0.f, 0.f, 0.f}, (f32x4){0.f, 0.f, 0.f, 0.f}};
    for (long p0 = p_begin; p0 < p_end; p0 += WG_KP) {
        // g tile: 32 pixels x 32 rows; thread t < 128: pixel t/4, rows (t%4)*8..+7
        if (tid < 128) {
            int pl = tid >> 2, rs = (tid & 3) * 8;
            long pix = p0 + pl;
            bf16x8 v = zero8();
            if (pix < p_end) {
                if (a.mode == G_CONV) {
                    if (r0 + rs < a.M) {
                        // g(row = co, p) = g[p][co], g grid = forward output grid
                        const bf16* src = a.g + pix * a.Cg + r0 + rs;
                        if (r0 + rs + 8 <= a.M) {
                            v = ld8(src);
                        } else {
                            for (int e = 0; e < 8 && r0 + rs + e < a.M; ++e) v[e] = src[e];
                        }
                    }
                } else {
                    // row = (2a+d)*Cg + co; p = (b, y, x) on the up-conv input grid
                    const Pix pp = pix_of(pix, a.Hi, a.Wi);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        int row = r0 + rs + e;
                        if (row >= a.M) break;
                        int ad = row / a.Cg, co = row - ad * a.Cg;
                        long gi = (((long)pp.b * a.Hg + 2 * pp.y + (ad >> 1)) * a.Wg + 2 * pp.x + (ad & 1)) * a.Cg + co;
                        v[e] = a.g[gi];
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) Ag[rs + e][pl] = v[e];
        }
        // x tile: 32 pixels x 64 k; thread t: pixel t/8, k (t%8)*8..+7
        {
            int pl = tid >> 3, ks = (tid & 7) * 8;
            long pix = p0 + pl;
            bf16x8 v = (pix < p_end && c0 + ks < a.N) ? wg_gather_x(a, pix, c0 + ks) : zero8();
#pragma unroll
            for (int e = 0; e < 8; ++e) Bx[ks + e][pl] = v[e];
        }
        __syncthreads();
        bf16x8 fb = *reinterpret_cast<const bf16x8*>(&Bx[wave * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 fa = *reinterpret_cast<const bf16x8*>(&Ag[i * 16 + (lane & 15)][(lane >> 4) * 8]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[i], 0, 0, 0);
        }
        __syncthreads();
    }
    float* part = a.part + (long)blockIdx.z * a.M * a.Npad;
    const int col = c0 + wave * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int row = r0 + i * 16 + (lane >> 4) * 4 + e;
            if (row < a.M && col < a.Npad) part[(long)row * a.Npad + col] = acc[i][e];
        }
}

int launch_wgrad(const WgradArgs& a, int nsplit, hipStream_t s) {
    dim3 grid((a.Npad + WG_BN - 1) / WG_BN, (a.M + WG_BM - 1) / WG_BM, nsplit);
    TIMED_LAUNCH("k_wgrad", s, k_wgrad, grid, dim3(256), 0, s, a);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

}  // namespace helm
