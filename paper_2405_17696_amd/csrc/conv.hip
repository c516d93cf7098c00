// Implicit-GEMM convolution kernels on the gfx950 BF16 matrix cores.
//
// One GEMM kernel serves the forward 3x3 convolutions (stride 1 or 2, one or
// two concatenated sources, fused bias / residual / ReLU), the 2x2 up-sampling
// convolutions, and both data gradients; a second kernel forms the weight
// gradients with the reduction over pixels split across workgroups.
//
// MFMA v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16] and D[4(l/16)+i][l%16], i = 0..3.  Every kernel here
// passes the weights as A and the pixels as B, so that the accumulators of a
// lane are four consecutive output channels of one pixel (vector stores).
#include <algorithm>
#include <map>
#include <mutex>

#include "conv.h"

namespace helm {

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Four consecutive BF16 values of a per-pixel bias map, widened.
__device__ __forceinline__ float4 bmap4(const bf16* p) {
    typedef __bf16 bf16x4m __attribute__((ext_vector_type(4)));
    const bf16x4m v = *reinterpret_cast<const bf16x4m*>(p);
    return make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}

// Pixel (b, y, x) of row m of a B x Ho x Wo grid.
struct Pix {
    int b, y, x;
};
// 32-bit unsigned divisions: every row index of these grids fits in 31 bits
// (the launchers reject larger grids), and 64-bit division is a long software
// sequence on the GPU.
__device__ __forceinline__ Pix pix_of(long m, int Ho, int Wo) {
    Pix p;
    const unsigned mu = (unsigned)m, hw = (unsigned)Ho * (unsigned)Wo;
    const unsigned b = mu / hw, r = mu - b * hw;
    const unsigned y = r / (unsigned)Wo;
    p.b = (int)b;
    p.y = (int)y;
    p.x = (int)(r - y * (unsigned)Wo);
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

typedef __bf16 bf16x4g __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2g __attribute__((ext_vector_type(2)));
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
    // one LDS buffer: the double-buffered A and B tiles, reused by the epilogue
    __shared__ __attribute__((aligned(16))) bf16 smem[2 * (BM + BN) * LDS_K];
    bf16 (*As)[BM][LDS_K] = reinterpret_cast<bf16 (*)[BM][LDS_K]>(smem);
    bf16 (*Bs)[BN][LDS_K] = reinterpret_cast<bf16 (*)[BN][LDS_K]>(smem + 2 * BM * LDS_K);
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
        work_atomic(wc, (unsigned long long)(2ull * mr * nr * (unsigned long long)a.kvalid));
    }
    // the tile's biases (per output channel; an up-convolution's column n uses bias n mod N/4)
    __shared__ __attribute__((aligned(16))) float bias_s[BN];
    if (tid < BN && (a.epi == E_FWD || a.epi == E_UPFWD)) {
        const int n = n0 + tid, nb = a.epi == E_UPFWD ? n % (a.N >> 2 > 0 ? a.N >> 2 : 1) : n;
        bias_s[tid] = a.bias && n < a.N ? a.bias[nb] : 0.f;
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
            for (int j = 0; j < WTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j], fa[i], acc[i][j], 0, 0, 0);
        if (kc + 1 < nchunk) {
            store_chunk(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue: the MFMA ran with the weights as A, so acc[i][j][e] holds
    // D[m = row tile i + l%16][n = column tile j + 4 (l/16) + e]: four consecutive
    // output channels of one pixel per lane.
    // Overwriting bf16 outputs go through LDS: each lane finishes and rounds its
    // four values into an LDS copy of the BM x BN tile, then every lane stores 16
    // contiguous bytes, so each output row leaves as whole lines (the direct
    // 8-byte stores spread over 16 pixels were partial-line writes).
    constexpr int SP = BN + 8;   // LDS row stride (bf16) of the output tile
    constexpr bool fits = sizeof(smem) >= (size_t)BM * SP * sizeof(bf16);
    const int cout_up = a.N >> 2;
    const bool staged = fits && a.out && !a.outf &&
                        ((a.epi == E_FWD && (a.N & 7) == 0) || (a.epi == E_UPFWD && (cout_up & 7) == 0));
    if (staged) {
        bf16* ot = smem;
        __syncthreads();   // every wave is done with the last chunk's tiles
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
            const int ml = wm * (BM / WGM) + i * 16 + (lane & 15);
            const long m = m0 + ml;
#pragma unroll
            for (int j = 0; j < WTN; ++j) {
                const int nl = wn * (BN / WGN) + j * 16 + (lane >> 4) * 4, n = n0 + nl;
                f32x4 v = acc[i][j];
                if (m < a.M && n < a.N) {
                    if (a.epi == E_FWD) {
                        const long pm = m % ((long)a.Ho * a.Wo);
                        const float4 bb =
                            a.bmap ? bmap4(a.bmap + pm * a.N + n) : *reinterpret_cast<const float4*>(bias_s + nl);
                        v[0] += bb.x;
                        v[1] += bb.y;
                        v[2] += bb.z;
                        v[3] += bb.w;
                        if (a.resid) {
                            const bf16x4g r = *reinterpret_cast<const bf16x4g*>(a.resid + m * a.N + n);
#pragma unroll
                            for (int e = 0; e < 4; ++e) v[e] += (float)r[e];
                        }
                    } else {
                        const float4 bb = *reinterpret_cast<const float4*>(bias_s + nl);
                        v[0] += bb.x;
                        v[1] += bb.y;
                        v[2] += bb.z;
                        v[3] += bb.w;
                    }
                    if (a.relu)
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                }
                bf16x4g o;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
                *reinterpret_cast<bf16x4g*>(ot + ml * SP + nl) = o;
            }
        }
        __syncthreads();
        constexpr int CPR = BN / 8;   // 16-byte chunks per tile row
        for (int k = tid; k < BM * CPR; k += 256) {
            const int ml = k / CPR, c = k - ml * CPR;
            const long m = m0 + ml;
            const int n = n0 + c * 8;
            if (m >= a.M || n >= a.N) continue;
            long o;
            if (a.epi == E_FWD) {
                o = m * a.N + n;
            } else {
                const Pix p = pix_of(m, a.Ho, a.Wo);
                const int ad = n / cout_up, co = n - ad * cout_up;
                o = (((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) * cout_up + co;
            }
            *reinterpret_cast<bf16x8*>(a.out + o) = *reinterpret_cast<const bf16x8*>(ot + ml * SP + c * 8);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
        const long m = m0 + wm * (BM / WGM) + i * 16 + (lane & 15);
        if (m >= a.M) continue;
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int n = n0 + wn * (BN / WGN) + j * 16 + (lane >> 4) * 4;
            if (n >= a.N) continue;
            f32x4 v = acc[i][j];
            if (a.epi == E_FWD) {
                const long pm = m % ((long)a.Ho * a.Wo);     // pixel within the sample (bmap index)
                if ((a.N & 3) == 0) {
                    const float4 bb = a.bmap ? bmap4(a.bmap + pm * a.N + n) : *reinterpret_cast<const float4*>(a.bias + n);
                    v[0] += bb.x;
                    v[1] += bb.y;
                    v[2] += bb.z;
                    v[3] += bb.w;
                    if (a.resid) {
                        const bf16x4g r = *reinterpret_cast<const bf16x4g*>(a.resid + m * a.N + n);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] += (float)r[e];
                    }
                    if (a.relu)
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                    if (a.out) {
                        bf16x4g o;
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
                        *reinterpret_cast<bf16x4g*>(a.out + m * a.N + n) = o;
                    }
                    if (a.outf) *reinterpret_cast<f32x4*>(a.outf + m * a.N + n) = v;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (n + e >= a.N) break;
                        float w = v[e] + (a.bmap ? (float)a.bmap[pm * a.N + n + e] : a.bias[n + e]);
                        if (a.resid) w += (float)a.resid[m * a.N + n + e];
                        if (a.relu) w = w > 0.f ? w : 0.f;
                        if (a.out) a.out[m * a.N + n + e] = (bf16)w;
                        if (a.outf) a.outf[m * a.N + n + e] = w;
                    }
                }
            } else if (a.epi == E_UPFWD) {
                const int cout = a.N >> 2;
                const Pix p = pix_of(m, a.Ho, a.Wo);
                if ((cout & 3) == 0) {
                    const int ad = n / cout, co = n - ad * cout;
                    const long o = (((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) *
                                       cout + co;
                    const float4 bb = *reinterpret_cast<const float4*>(a.bias + co);
                    v[0] += bb.x;
                    v[1] += bb.y;
                    v[2] += bb.z;
                    v[3] += bb.w;
                    bf16x4g ov;
#pragma unroll
                    for (int e = 0; e < 4; ++e) ov[e] = (bf16)(a.relu ? (v[e] > 0.f ? v[e] : 0.f) : v[e]);
                    *reinterpret_cast<bf16x4g*>(a.out + o) = ov;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ne = n + e;
                        if (ne >= a.N) break;
                        const int ad = ne / cout, co = ne - ad * cout;
                        const long o =
                            (((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) * cout + co;
                        float w = v[e] + a.bias[co];
                        if (a.relu) w = w > 0.f ? w : 0.f;
                        a.out[o] = (bf16)w;
                    }
                }
            } else {  // E_ACC
                const int n2 = a.N - a.n1;
                if (n + 4 <= a.n1 && (a.n1 & 3) == 0) {
                    f32x4* q = reinterpret_cast<f32x4*>(a.acc1 + m * a.n1 + n);
                    *q = *q + v;
                } else if (n >= a.n1 && n + 4 <= a.N && (n2 & 3) == 0 && ((n - a.n1) & 3) == 0) {
                    f32x4* q = reinterpret_cast<f32x4*>(a.acc2 + m * n2 + (n - a.n1));
                    *q = *q + v;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ne = n + e;
                        if (ne >= a.N) break;
                        if (ne < a.n1)
                            a.acc1[m * a.n1 + ne] += v[e];
                        else
                            a.acc2[m * n2 + (ne - a.n1)] += v[e];
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ halo-tiled 3x3 stride-1 convolution
// A block computes 16 x 16 output pixels of one sample for BN output channels.
// Per chunk of 32 input channels it stages the 18 x 18 input patch and the nine
// taps of the weights in LDS once and runs all nine taps from there (the
// implicit-GEMM kernel above re-reads every input pixel nine times through L2).
// Wave w owns output rows 4w .. 4w+3; for a fixed kx the six patch rows
// 4w .. 4w+5 each feed up to three (row, ky) products, so every pixel
// fragment is read from LDS once per kx instead of once per tap.
// The MFMA takes the weights as A and the pixels as B, so a lane ends with four
// consecutive output channels of one pixel and stores them as one 8-byte vector.
// FLIP = 1 runs the data gradient of a stride-1 convolution: taps mirrored,
// weights [Cin][tap][Cout].
constexpr int HT = 16;              // tile edge (pixels)
constexpr int HP = HT + 2;          // patch edge
constexpr int HC = 32;              // channels per chunk
constexpr int HLD = HC + 8;         // padded LDS row (bf16)
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

typedef unsigned u32x4s __attribute__((ext_vector_type(4)));
// 16-byte raw buffer load; an offset at or past the descriptor's byte count reads zeros.
__device__ __forceinline__ bf16x8 bload8(__amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return __builtin_bit_cast(bf16x8, v);
}
// Raw buffer descriptor over nbytes at p (dword data format, no stride).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* p, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

// ------------------------------------------------------------------ implicit GEMM, deeper prefetch
// The implicit GEMM above keeps one 32-deep chunk of A and B in flight.  At the
// stride-2 layers a chunk holds only 4 to 8 MFMAs per wave and every chunk waits
// for its own loads, so a block costs about one load latency per chunk.  This
// form keeps GPF_D chunks in flight in registers.  It serves forward 3 x 3
// convolutions (any stride) whose sources have multiples of 32 channels: a chunk
// then lies within one tap and one source, so tap, source and channel offset are
// the same for the whole chunk, and each thread decodes its pixels once.  Every
// load is a raw buffer load, a fixed number per chunk (a read outside the image,
// past M or past N gets an offset past the buffer, which reads zeros), so the
// wait before a chunk's LDS store covers that chunk's loads only.  The sums run
// over K in the order of k_gemm, so the two give the same results.
constexpr int GPF_D = 3;                   // chunks in flight: divides 9, 18 and 36 (C = 32, 64, 128)
constexpr unsigned GPF_OOR = 0x80000000u;  // an offset no descriptor here reaches (byte counts < 2^31)
template <int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void k_gemm_pf(GemmArgs a, unsigned long long* wc) {
    constexpr int WTM = BM / WGM / 16, WTN = BN / WGN / 16;
    constexpr int ASEG = BM * KC / 8, BSEG = BN * KC / 8;
    constexpr int APT = (ASEG + 255) / 256, BPT = (BSEG + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 smem[2 * (BM + BN) * LDS_K];
    bf16 (*As)[BM][LDS_K] = reinterpret_cast<bf16 (*)[BM][LDS_K]>(smem);
    bf16 (*Bs)[BN][LDS_K] = reinterpret_cast<bf16 (*)[BN][LDS_K]>(smem + 2 * BM * LDS_K);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const long m0 = (long)blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    const int nchunk = a.K / KC;   // a multiple of GPF_D (checked by the launcher)
    if (a.st && ((long)a.Ho * a.Wo) % BM == 0) {
        // a tile never straddles two samples when Ho*Wo is a multiple of BM
        const int b = (int)(m0 / ((long)a.Ho * a.Wo));
        const RhsState& S = a.st[a.rhs0 + b];
        if (!S.active || S.cycdone) return;
    }
    if (wc && tid == 0) {
        long mr = a.M - m0 < BM ? a.M - m0 : BM;
        int nr = a.N - n0 < BN ? a.N - n0 : BN;
        work_atomic(wc, (unsigned long long)(2ull * mr * nr * (unsigned long long)a.kvalid));
    }
    __shared__ __attribute__((aligned(16))) float bias_s[BN];
    if (tid < BN) bias_s[tid] = a.bias && n0 + tid < a.N ? a.bias[n0 + tid] : 0.f;

    // per thread: the pixel of each A segment (source element offsets of its sample,
    // top-left input position of its 3 x 3 window) and the weight row of each B segment
    int ay[APT], ax[APT];
    unsigned ab1[APT], ab2[APT], asub[APT];
    bool arow[APT];
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const int sg = tid + q * 256, row = sg >> 2;
        const long m = m0 + row;
        arow[q] = sg < ASEG && m < a.M;
        const Pix p = pix_of(arow[q] ? m : 0, a.Ho, a.Wo);
        ay[q] = p.y * a.stride - 1;
        ax[q] = p.x * a.stride - 1;
        ab1[q] = (unsigned)((long)p.b * a.abs1);
        ab2[q] = (unsigned)((long)p.b * a.abs2);
        asub[q] = (unsigned)((sg & 3) * 8);
    }
    unsigned boff[BPT];
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        const int sg = tid + q * 256, n = n0 + (sg >> 2);
        boff[q] = sg < BSEG && n < a.N ? (unsigned)(((long)n * a.K + (sg & 3) * 8) * 2) : GPF_OOR;
    }
    const long s1n = a.abs1 ? (long)a.B * a.abs1 : (long)a.Hi * a.Wi * a.c1;
    const long s2n = a.c2 ? (a.abs2 ? (long)a.B * a.abs2 : (long)a.Hi * a.Wi * a.c2) : 0;
    const __amdgpu_buffer_rsrc_t rs1 = brsrc(a.a1, (unsigned)(s1n * 2));
    const __amdgpu_buffer_rsrc_t rs2 = brsrc(a.c2 ? a.a2 : a.a1, (unsigned)((a.c2 ? s2n : s1n) * 2));
    const __amdgpu_buffer_rsrc_t rsw = brsrc(a.w, (unsigned)((long)a.N * a.K * 2));
    const int C = a.c1 + a.c2;

    // loads of chunk kc (none past the last chunk: every offset out of range)
    struct Set {
        bf16x8 a[APT], b[BPT];
    };
    auto issue = [&](int kc) -> Set {
        Set r;
        const bool live = kc < nchunk;
        const int k0 = kc * KC;
        const int tap = k0 / C, c0 = k0 - tap * C;
        const int ky = tap / 3, kx = tap - ky * 3;
        const bool src2 = c0 >= a.c1;
        const int cs = src2 ? a.c2 : a.c1, cc = src2 ? c0 - a.c1 : c0;
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const int yi = ay[q] + ky, xi = ax[q] + kx;
            const bool ok = live && arow[q] && (unsigned)yi < (unsigned)a.Hi && (unsigned)xi < (unsigned)a.Wi;
            const unsigned off =
                ok ? ((src2 ? ab2[q] : ab1[q]) + (unsigned)((yi * a.Wi + xi) * cs + cc) + asub[q]) * 2u : GPF_OOR;
            r.a[q] = bload8(src2 ? rs2 : rs1, off);
        }
#pragma unroll
        for (int q = 0; q < BPT; ++q)
            r.b[q] = bload8(rsw, live && boff[q] != GPF_OOR ? boff[q] + (unsigned)k0 * 2u : GPF_OOR);
        return r;
    };
    auto store = [&](int buf, const Set& r) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const int sg = tid + q * 256;
            if (sg < ASEG) *reinterpret_cast<bf16x8*>(&As[buf][sg >> 2][(sg & 3) * 8]) = r.a[q];
        }
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int sg = tid + q * 256;
            if (sg < BSEG) *reinterpret_cast<bf16x8*>(&Bs[buf][sg >> 2][(sg & 3) * 8]) = r.b[q];
        }
    };
    f32x4 acc[WTM][WTN];
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    auto mma = [&](int buf) {
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
            for (int j = 0; j < WTN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j], fa[i], acc[i][j], 0, 0, 0);
    };

    // chunk c is multiplied from LDS buffer c & 1; three register sets hold the next
    // chunks, each refilled GPF_D chunks ahead as soon as its chunk is in LDS
    Set r0 = issue(0), r1 = issue(1), r2 = issue(2);
    store(0, r0);
    __syncthreads();
    for (int kc = 0; kc < nchunk; kc += GPF_D) {
        r0 = issue(kc + 3);
        mma(kc & 1);
        store((kc + 1) & 1, r1);
        __syncthreads();
        r1 = issue(kc + 4);
        mma((kc + 1) & 1);
        store(kc & 1, r2);
        __syncthreads();
        r2 = issue(kc + 5);
        mma(kc & 1);
        if (kc + 3 < nchunk) {
            store((kc + 1) & 1, r0);
            __syncthreads();
        }
    }

    // epilogue through LDS, as in k_gemm's forward path: each lane finishes its four
    // channels of one pixel into an LDS copy of the tile, then whole 16-byte rows
    constexpr int SP = BN + 8;
    static_assert(sizeof(smem) >= (size_t)BM * SP * sizeof(bf16), "epilogue tile");
    bf16* ot = smem;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
        const int ml = wm * (BM / WGM) + i * 16 + (lane & 15);
        const long m = m0 + ml;
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int nl = wn * (BN / WGN) + j * 16 + (lane >> 4) * 4, n = n0 + nl;
            f32x4 v = acc[i][j];
            if (m < a.M && n < a.N) {
                const long pm = m % ((long)a.Ho * a.Wo);
                const float4 bb =
                    a.bmap ? bmap4(a.bmap + pm * a.N + n) : *reinterpret_cast<const float4*>(bias_s + nl);
                v[0] += bb.x;
                v[1] += bb.y;
                v[2] += bb.z;
                v[3] += bb.w;
                if (a.resid) {
                    const bf16x4g r = *reinterpret_cast<const bf16x4g*>(a.resid + m * a.N + n);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += (float)r[e];
                }
                if (a.relu)
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                if (a.outf) *reinterpret_cast<f32x4*>(a.outf + m * a.N + n) = v;   // FP32 copy (layer tests)
            }
            bf16x4g o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
            *reinterpret_cast<bf16x4g*>(ot + ml * SP + nl) = o;
        }
    }
    __syncthreads();
    constexpr int CPR = BN / 8;
    for (int k = tid; k < BM * CPR; k += 256) {
        const int ml = k / CPR, c = k - ml * CPR;
        const long m = m0 + ml;
        const int n = n0 + c * 8;
        if (m >= a.M || n >= a.N) continue;
        *reinterpret_cast<bf16x8*>(a.out + m * a.N + n) = *reinterpret_cast<const bf16x8*>(ot + ml * SP + c * 8);
    }
}

// Register staging of one 32-channel chunk of a tile's patch (and of the nine
// taps of BN output channels' weights).  The per-thread byte offsets of its
// segments are computed once per tile (and input half) and once per block for
// the weights; a chunk's loads then only add the channel offset.  Patch pixels
// outside the image and weight rows past N get an offset past the end of their
// buffer, so the buffer loads return zeros without a branch.
template <int BN>
struct HaloStage {
    static constexpr int PSEG = HP * HP * (HC / 8);   // 16-byte segments of the patch
    static constexpr int WSEG = 9 * BN * (HC / 8);    // and of the weights
    static constexpr int PPT = (PSEG + 255) / 256, WPT = (WSEG + 255) / 256;
    bf16x8 rp[PPT], rw[WPT];
    unsigned po[PPT], wo[WPT];
    __amdgpu_buffer_rsrc_t rs_p, rs_w;
    int half = -1;   // input half the patch offsets refer to (0: a1, 1: a2)

    // Patch offsets of the 16 x 16 tile at (ty0, tx0) of sample b in input half s2.
    __device__ __forceinline__ void tile(const GemmArgs& a, int tid, int b, int ty0, int tx0, int s2) {
        const bf16* src = s2 ? a.a2 + b * a.abs2 : a.a1 + b * a.abs1;
        const int cs = s2 ? a.c2 : a.c1;
        const unsigned nrec = (unsigned)a.Hi * (unsigned)a.Wi * (unsigned)cs * 2u;
        rs_p = brsrc(src, nrec);
        half = s2;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int sg = tid + q * 256;
            const int pix = sg >> 2, sub = sg & 3;
            const int py = pix / HP, px = pix - py * HP;
            const int yi = ty0 + py - 1, xi = tx0 + px - 1;
            const bool in = sg < PSEG && (unsigned)yi < (unsigned)a.Hi && (unsigned)xi < (unsigned)a.Wi;
            po[q] = in ? ((unsigned)(yi * a.Wi + xi) * (unsigned)cs + (unsigned)(sub * 8)) * 2u : nrec;
        }
    }
    // Weight offsets of output channels n0 .. n0 + BN - 1 (rows [N][K], K = 9 C tap-major).
    __device__ __forceinline__ void wset(const GemmArgs& a, int tid, int n0) {
        const unsigned nrec = (unsigned)a.N * (unsigned)a.K * 2u;
        rs_w = brsrc(a.w, nrec);
        const int C = a.c1 + a.c2;
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int sg = tid + q * 256;
            const int row = sg >> 2, sub = sg & 3;   // row = tap * BN + n
            const int tap = row / BN, n = row - tap * BN;
            wo[q] = sg < WSEG && n0 + n < a.N ? (unsigned)((n0 + n) * a.K + tap * C + sub * 8) * 2u : nrec;
        }
    }
    // Chunk at absolute input channel c0 (the patch offsets must refer to its half).
    __device__ __forceinline__ void issue(const GemmArgs& a, int tid, int c0, bool weights) {
        const unsigned cc = (unsigned)(half ? c0 - a.c1 : c0) * 2u;
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            if (tid + q * 256 < PSEG) rp[q] = bload8(rs_p, po[q] + cc);
        if (!weights) return;
#pragma unroll
        for (int q = 0; q < WPT; ++q)
            if (tid + q * 256 < WSEG) rw[q] = bload8(rs_w, wo[q] + (unsigned)c0 * 2u);
    }
    // All in one: offsets for this tile (and weights), then the loads.
    __device__ __forceinline__ void load(const GemmArgs& a, int tid, int b, int ty0, int tx0, int n0, int c0,
                                         bool weights) {
        tile(a, tid, b, ty0, tx0, c0 >= a.c1);
        if (weights) wset(a, tid, n0);
        issue(a, tid, c0, weights);
    }
    template <int WLD>
    __device__ __forceinline__ void store(bf16 (*Ps)[HLD], bf16 (*Ws)[BN][WLD], int tid, bool weights) const {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int sg = tid + q * 256;
            if (sg >= PSEG) break;
            *reinterpret_cast<bf16x8*>(&Ps[sg >> 2][(sg & 3) * 8]) = rp[q];
        }
        if (!weights) return;
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int sg = tid + q * 256;
            if (sg >= WSEG) break;
            const int row = sg >> 2;
            *reinterpret_cast<bf16x8*>(&Ws[row / BN][row % BN][(sg & 3) * 8]) = rw[q];
        }
    }
};

// acc[i][j] += sum over the 9 taps and the staged 32 channels.  With 32 output
// channels the three kernel rows' weight fragments are held for a fixed kx and
// each pixel fragment is read once; with 64 the register budget (occupancy 2)
// allows only the tap-by-tap order.
template <int BN, int FLIP, int WLD = HLD>
__device__ __forceinline__ void halo_mma(const bf16 (*Ps)[HLD], const bf16 (*Ws)[BN][WLD], int coff,
                                         f32x4 (&acc)[4][BN / 16], int lane, int wave) {
    constexpr int WTN = BN / 16;
    if constexpr (BN <= 32) {
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            bf16x8 fw[3][WTN];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int tap = FLIP ? 8 - (3 * ky + kx) : 3 * ky + kx;
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    fw[ky][j] =
                        *reinterpret_cast<const bf16x8*>(&Ws[tap][j * 16 + (lane & 15)][coff + (lane >> 4) * 8]);
            }
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const bf16x8 fx =
                    *reinterpret_cast<const bf16x8*>(&Ps[(wave * 4 + r) * HP + (lane & 15) + kx][(lane >> 4) * 8]);
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) {
                    const int i = r - ky;          // output row 4w + i reads patch row 4w + i + ky
                    if (i < 0 || i > 3) continue;
#pragma unroll
                    for (int j = 0; j < WTN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[ky][j], fx, acc[i][j], 0, 0, 0);
                }
            }
        }
    } else {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = FLIP ? 2 - tap / 3 : tap / 3, kx = FLIP ? 2 - tap % 3 : tap % 3;
            bf16x8 fw[WTN];
#pragma unroll
            for (int j = 0; j < WTN; ++j)
                fw[j] = *reinterpret_cast<const bf16x8*>(&Ws[tap][j * 16 + (lane & 15)][coff + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bf16x8 fx = *reinterpret_cast<const bf16x8*>(
                    &Ps[(wave * 4 + i + ky) * HP + (lane & 15) + kx][(lane >> 4) * 8]);
#pragma unroll
                for (int j = 0; j < WTN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fx, acc[i][j], 0, 0, 0);
            }
        }
    }
}

// acc[i][j][e] = D[n = n0 + 16 j + 4 (l/16) + e][pixel (ty0 + 4w + i, tx0 + l%16)]
template <int BN, int EPI>
__device__ __forceinline__ void halo_epilogue(const GemmArgs& a, const f32x4 (&acc)[4][BN / 16], int b, int ty0,
                                              int tx0, int n0, int lane, int wave) {
    constexpr int WTN = BN / 16;
    const int x = tx0 + (lane & 15);
    if (x >= a.Wo) return;
    const bool vec = (a.N & 3) == 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ty0 + wave * 4 + i;
        if (y >= a.Ho) continue;
        const long m = ((long)b * a.Ho + y) * a.Wo + x;
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int n = n0 + j * 16 + (lane >> 4) * 4;
            if (n >= a.N) continue;
            f32x4 v = acc[i][j];
            if (EPI == E_FWD) {
                if (vec) {
                    const float4 bb = a.bmap ? bmap4(a.bmap + ((long)y * a.Wo + x) * a.N + n)
                                             : *reinterpret_cast<const float4*>(a.bias + n);
                    v[0] += bb.x;
                    v[1] += bb.y;
                    v[2] += bb.z;
                    v[3] += bb.w;
                    if (a.resid) {
                        const bf16x4 r = *reinterpret_cast<const bf16x4*>(a.resid + m * a.N + n);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] += (float)r[e];
                    }
                    if (a.relu)
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                    if (a.out) {
                        bf16x4 o;
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
                        *reinterpret_cast<bf16x4*>(a.out + m * a.N + n) = o;
                    }
                    if (a.outf) *reinterpret_cast<f32x4*>(a.outf + m * a.N + n) = v;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (n + e >= a.N) break;
                        float w = v[e] + (a.bmap ? (float)a.bmap[((long)y * a.Wo + x) * a.N + n + e] : a.bias[n + e]);
                        if (a.resid) w += (float)a.resid[m * a.N + n + e];
                        if (a.relu) w = w > 0.f ? w : 0.f;
                        if (a.out) a.out[m * a.N + n + e] = (bf16)w;
                        if (a.outf) a.outf[m * a.N + n + e] = w;
                    }
                }
            } else {  // E_ACC
                const int n2 = a.N - a.n1;
                if (n + 4 <= a.n1 && (a.n1 & 3) == 0) {
                    f32x4* p = reinterpret_cast<f32x4*>(a.acc1 + m * a.n1 + n);
                    *p = *p + v;
                } else if (n >= a.n1 && n + 4 <= a.N && (n2 & 3) == 0 && ((n - a.n1) & 3) == 0) {
                    f32x4* p = reinterpret_cast<f32x4*>(a.acc2 + m * n2 + (n - a.n1));
                    *p = *p + v;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ne = n + e;
                        if (ne >= a.N) break;
                        if (ne < a.n1)
                            a.acc1[m * a.n1 + ne] += v[e];
                        else
                            a.acc2[m * n2 + (ne - a.n1)] += v[e];
                    }
                }
            }
        }
    }
}

// Forward epilogue through LDS: each lane finishes its accumulators as above
// (bias or bias map, ReLU, rounding to bf16) but writes them to an LDS copy of
// the block's 16 x 16 x BN output tile; after a barrier every lane
// stores 16 contiguous bytes, so a pixel's BN channels leave as whole 64- or
// 128-byte lines in one instruction instead of four 8-byte pieces per lane
// spread over 16 pixels (partial-line writes ran at under 2 TB/s).  scratch
// holds 256 (BN + 8) bf16; bias_s holds the block's BN biases (staged into LDS
// at the start of the kernel, so the epilogue does not wait on a global load);
// every thread of the block must call this.
template <int BN>
__device__ __forceinline__ bool halo_lds_epilogue_ok(const GemmArgs& a) {
    return a.out && !a.outf && (a.N & 7) == 0;
}
template <int BN>
__device__ __forceinline__ void halo_epilogue_lds(const GemmArgs& a, const f32x4 (&acc)[4][BN / 16], int b, int ty0,
                                                  int tx0, int n0, int tid, bf16* scratch, const float* bias_s) {
    constexpr int WTN = BN / 16, SP = BN + 8;   // LDS pixel stride (bf16), 16-byte aligned rows
    const int lane = tid & 63, wave = tid >> 6;
    const int x = tx0 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ty0 + wave * 4 + i;
        const bool in = x < a.Wo && y < a.Ho;
        const long m = ((long)b * a.Ho + y) * a.Wo + x;
        const int p = (wave * 4 + i) * HT + (lane & 15);
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
            const int nl = j * 16 + (lane >> 4) * 4, n = n0 + nl;
            f32x4 v = acc[i][j];
            if (in && n < a.N) {
                const float4 bb = a.bmap ? bmap4(a.bmap + ((long)y * a.Wo + x) * a.N + n)
                                         : *reinterpret_cast<const float4*>(bias_s + nl);
                v[0] += bb.x;
                v[1] += bb.y;
                v[2] += bb.z;
                v[3] += bb.w;
                if (a.relu && !a.resid)
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
            }
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
            *reinterpret_cast<bf16x4*>(scratch + p * SP + nl) = o;
        }
    }
    __syncthreads();
    // a residual is added here on whole 16-byte rows: convolution plus bias is rounded to bf16
    // above, the sum with the residual is rounded again
    // every thread issues CPP stores (pixels outside the image are written past the end of the
    // output, which the buffer's range check drops): with a fixed count the persistent kernels'
    // wait for their next tile's prefetched loads need not wait for these stores as well
    constexpr int CPP = BN / 8;                   // 16-byte chunks per pixel
    const unsigned nrec = (unsigned)((long)a.B * a.Ho * a.Wo * a.N * 2);
    const __amdgpu_buffer_rsrc_t ro = brsrc(a.out, nrec);
#pragma unroll
    for (int r = 0; r < CPP; ++r) {
        const int k = tid + r * 256;
        const int p = k / CPP, c = k - p * CPP;
        const int y = ty0 + p / HT, xx = tx0 + (p & (HT - 1)), n = n0 + c * 8;
        const bool ok = y < a.Ho && xx < a.Wo && n < a.N;
        const unsigned off = ok ? (unsigned)(((((long)b * a.Ho + y) * a.Wo + xx) * a.N + n) * 2) : nrec;
        bf16x8 t = *reinterpret_cast<const bf16x8*>(scratch + p * SP + c * 8);
        if (a.resid) {
            const bf16x8 rr = bload8(brsrc(a.resid, nrec), off);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float w = (float)t[e] + (float)rr[e];
                if (a.relu) w = w > 0.f ? w : 0.f;
                t[e] = (bf16)w;
            }
        }
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4s, t), ro, off, 0, 0);
    }
    __syncthreads();
}

__device__ __forceinline__ unsigned long long halo_work(const GemmArgs& a, int ty0, int tx0, int n0, int bn) {
    const int my = a.Ho - ty0 < HT ? a.Ho - ty0 : HT, mx = a.Wo - tx0 < HT ? a.Wo - tx0 : HT;
    const int nr = a.N - n0 < bn ? a.N - n0 : bn;
    return 2ull * my * mx * nr * (unsigned long long)(9 * (a.c1 + a.c2));
}
__device__ __forceinline__ void halo_count(const GemmArgs& a, unsigned long long* wc, int ty0, int tx0, int n0,
                                           int bn) {
    if (wc) work_atomic(wc, halo_work(a, ty0, tx0, n0, bn));
}

// One tile per block; the next chunk's patch and weights are prefetched into
// registers while the current chunk runs.
template <int BN, int FLIP, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BN <= 32 ? 3 : 2))) void k_conv3_halo(GemmArgs a, unsigned long long* wc) {
    constexpr int WTN = BN / 16;
    __shared__ __attribute__((aligned(16))) bf16 Ps[HP * HP][HLD];
    __shared__ __attribute__((aligned(16))) bf16 Ws[9][BN][HLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (a.Wo + HT - 1) / HT, tiles_y = (a.Ho + HT - 1) / HT;
    int t = blockIdx.x;
    const int tx0 = (t % tiles_x) * HT;
    t /= tiles_x;
    const int ty0 = (t % tiles_y) * HT;
    const int b = t / tiles_y;
    const int n0 = blockIdx.y * BN;
    if (a.st && !(a.st[a.rhs0 + b].active && !a.st[a.rhs0 + b].cycdone)) return;
    if (tid == 0) halo_count(a, wc, ty0, tx0, n0, BN);
    __shared__ __attribute__((aligned(16))) float bias_s[BN];
    if (EPI == E_FWD && tid < BN) bias_s[tid] = a.bias && n0 + tid < a.N ? a.bias[n0 + tid] : 0.f;
    f32x4 acc[4][WTN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    HaloStage<BN> st;
    const int nchunk = (a.c1 + a.c2) / HC;
    st.load(a, tid, b, ty0, tx0, n0, 0, true);
    for (int ch = 0; ch < nchunk; ++ch) {
        st.store(Ps, Ws, tid, true);
        __syncthreads();
        if (ch + 1 < nchunk) {
            const int c0 = (ch + 1) * HC;
            if (c0 == a.c1) st.tile(a, tid, b, ty0, tx0, 1);
            st.issue(a, tid, c0, true);
        }
        halo_mma<BN, FLIP>(Ps, Ws, 0, acc, lane, wave);
        __syncthreads();
    }
    static_assert(sizeof(Ws) >= 256 * (BN + 8) * sizeof(bf16), "epilogue scratch");
    if (EPI == E_FWD && halo_lds_epilogue_ok<BN>(a))
        halo_epilogue_lds<BN>(a, acc, b, ty0, tx0, n0, tid, &Ws[0][0][0], bias_s);
    else
        halo_epilogue<BN, EPI>(a, acc, b, ty0, tx0, n0, lane, wave);
}

// ------------------------------------------------------------------ double-buffered wide-tile halo kernel
// One 16 x 32 output tile and BN = 64 output channels per 512-thread block.
// Each 32-channel chunk of the 18 x 34 input patch and the chunk's nine taps of
// weights go straight from memory into LDS with 16-byte buffer loads (lane l of
// a load instruction lands at byte 16 l of its 1 KB destination, so the dense
// [pixel][32 channel] layout needs no register staging; out-of-image pixels and
// weight rows past N are read past the end of their buffer and arrive as zeros).
// Two LDS stages alternate: while the eight waves multiply chunk c out of one
// stage, the loads of chunk c + 1 fill the other, so a chunk costs one barrier.
// The 512-pixel tile halves the weight traffic per output of a 16 x 16 tile.
// Wave w owns output rows 4 (w & 3) .. + 3 of column half w >> 2.
constexpr int DTY = 16, DTX = 32;                 // output tile
constexpr int DPY = DTY + 2, DPX = DTX + 2;       // input patch
constexpr int DPSEG = DPY * DPX * 4;              // 16-byte segments of one patch chunk (2448)
constexpr int DWSEG = 9 * 64 * 4;                 // and of one weight chunk (2304)
constexpr int DPINS = (DPSEG + 63) / 64;          // wave-wide load instructions per patch chunk (39)
constexpr int DWINS = DWSEG / 64;                 // per weight chunk (36)
constexpr int DPPT = (DPINS + 7) / 8, DWPT = (DWINS + 7) / 8;   // per wave (5, 5)
constexpr int DPBYTES = DPINS * 1024;             // patch region of a stage (the last load's
                                                  // lanes past the patch write zeros into its tail)
constexpr int DSTAGE = DPBYTES + DWINS * 1024;    // bytes per LDS stage (76800)
typedef __attribute__((address_space(3))) void lds_void_t;

struct DlStage {
    unsigned po[DPPT];   // per-lane byte offsets of this wave's patch segments (past the range: zeros)
    unsigned wo[DWPT];   // and of its weight segments

    // Patch offsets of the tile at (ty0, tx0) in input half s2 (0: a1, 1: a2).
    __device__ __forceinline__ void tile(const GemmArgs& a, int lane, int wave, int ty0, int tx0, int s2) {
        const int cs = s2 ? a.c2 : a.c1;
        const unsigned nrec = (unsigned)a.Hi * (unsigned)a.Wi * (unsigned)cs * 2u;
#pragma unroll
        for (int q = 0; q < DPPT; ++q) {
            const int sg = (wave + 8 * q) * 64 + lane;
            const int pix = sg >> 2, sub = sg & 3;
            const int py = pix / DPX, px = pix - py * DPX;
            const int yi = ty0 + py - 1, xi = tx0 + px - 1;
            const bool in = sg < DPSEG && (unsigned)yi < (unsigned)a.Hi && (unsigned)xi < (unsigned)a.Wi;
            po[q] = in ? ((unsigned)(yi * a.Wi + xi) * (unsigned)cs + (unsigned)(sub * 8)) * 2u : nrec;
        }
    }
    __device__ __forceinline__ void wset(const GemmArgs& a, int lane, int wave, int n0) {
        const unsigned nrec = (unsigned)a.N * (unsigned)a.K * 2u;
        const int C = a.c1 + a.c2;
#pragma unroll
        for (int q = 0; q < DWPT; ++q) {
            const int sg = (wave + 8 * q) * 64 + lane;   // row = tap * 64 + n
            const int row = sg >> 2, sub = sg & 3;
            const int tap = row >> 6, n = row & 63;
            wo[q] = sg < DWSEG && n0 + n < a.N ? (unsigned)((n0 + n) * a.K + tap * C + sub * 8) * 2u : nrec;
        }
    }
    // Loads of sample b's chunk at absolute input channel c0 into the stage at st (bytes); the
    // patch offsets must refer to the chunk's input half.
    __device__ __forceinline__ void issue(const GemmArgs& a, int wave, int b, int c0, unsigned char* st) const {
        const bool s2 = c0 >= a.c1;
        const bf16* src = s2 ? a.a2 + b * a.abs2 : a.a1 + b * a.abs1;
        const unsigned nrec = (unsigned)a.Hi * (unsigned)a.Wi * (unsigned)(s2 ? a.c2 : a.c1) * 2u;
        const __amdgpu_buffer_rsrc_t rs_p = brsrc(src, nrec);
        const __amdgpu_buffer_rsrc_t rs_w = brsrc(a.w, (unsigned)a.N * (unsigned)a.K * 2u);
        const unsigned cc = (unsigned)(s2 ? c0 - a.c1 : c0) * 2u;
#pragma unroll
        for (int q = 0; q < DPPT; ++q) {
            const int ins = wave + 8 * q;
            if (ins < DPINS)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_p, (lds_void_t*)(st + ins * 1024), 16, po[q] + cc, 0, 0, 0);
        }
        unsigned char* ws = st + DPBYTES;
#pragma unroll
        for (int q = 0; q < DWPT; ++q) {
            const int ins = wave + 8 * q;
            if (ins < DWINS)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_w, (lds_void_t*)(ws + ins * 1024), 16, wo[q] + (unsigned)c0 * 2u,
                                                         0, 0, 0);
        }
    }
};

// acc[i][j] += one staged chunk; P = [DPY*DPX][32], W = [9][64][32] (bf16).
// Tap by tap, with the next tap's eight fragments (four weight rows, four patch
// rows) read from LDS before the current tap's sixteen MFMAs are issued: a wave
// hides its own LDS latency behind a whole tap.  The scheduling barriers keep
// the compiler from sinking the reads next to their uses.
__device__ __forceinline__ void dl_mma(const bf16* P, const bf16* W, f32x4 (&acc)[4][4], int lane, int rg, int cx) {
    const int g8 = (lane >> 4) * 8;
    const bf16* pw = W + (lane & 15) * 32 + g8;
    const bf16* pp = P + ((rg * 4) * DPX + cx * 16 + (lane & 15)) * 32 + g8;
    bf16x8 fw[2][4], fx[2][4];
    auto fetch = [&](int tap, int buf) {
        const int ky = tap / 3, kx = tap % 3;
#pragma unroll
        for (int j = 0; j < 4; ++j) fw[buf][j] = *reinterpret_cast<const bf16x8*>(pw + (tap * 64 + j * 16) * 32);
#pragma unroll
        for (int i = 0; i < 4; ++i) fx[buf][i] = *reinterpret_cast<const bf16x8*>(pp + ((i + ky) * DPX + kx) * 32);
    };
    fetch(0, 0);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int cur = tap & 1;
        if (tap + 1 < 9) fetch(tap + 1, cur ^ 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[cur][j], fx[cur][i], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Epilogue of one 16 x 32 tile (E_FWD).  With bf16 output and N a multiple of 8
// the accumulators go through the LDS scratch sc (>= 512 * 72 bf16, free when
// called; every thread of the block must call this): bias or bias map, ReLU when
// there is no residual, rounding to bf16, then whole 16-byte channel groups per
// store with the residual added on them.  Otherwise a per-element register path.
__device__ __forceinline__ void dl_epilogue(const GemmArgs& a, const f32x4 (&acc)[4][4], int b, int ty0, int tx0,
                                            int n0, int tid, bf16* sc, const float* bias_s) {
    const int lane = tid & 63, wave = tid >> 6, rg = wave & 3, cx = wave >> 2;
    const int x = tx0 + cx * 16 + (lane & 15);
    if ((a.N & 7) == 0 && a.out && !a.outf) {
        constexpr int SP = 64 + 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int py = rg * 4 + i, y = ty0 + py;
            const bool in = x < a.Wo && y < a.Ho;
            const int p = py * DTX + cx * 16 + (lane & 15);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int nl = j * 16 + (lane >> 4) * 4, n = n0 + nl;
                f32x4 v = acc[i][j];
                if (in && n < a.N) {
                    const float4 bb = a.bmap ? bmap4(a.bmap + ((long)y * a.Wo + x) * a.N + n)
                                             : *reinterpret_cast<const float4*>(bias_s + nl);
                    v[0] += bb.x;
                    v[1] += bb.y;
                    v[2] += bb.z;
                    v[3] += bb.w;
                    if (a.relu && !a.resid)
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                }
                bf16x4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
                *reinterpret_cast<bf16x4*>(sc + p * SP + nl) = o;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < DTY * DTX * 8 / 512; ++r) {
            const int k = tid + r * 512;
            const int p = k >> 3, c = k & 7;
            const int y = ty0 + p / DTX, xx = tx0 + p % DTX, n = n0 + c * 8;
            if (y < a.Ho && xx < a.Wo && n < a.N) {
                const long o = (((long)b * a.Ho + y) * a.Wo + xx) * a.N + n;
                bf16x8 v = *reinterpret_cast<const bf16x8*>(sc + p * SP + c * 8);
                if (a.resid) {
                    const bf16x8 rr = *reinterpret_cast<const bf16x8*>(a.resid + o);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        float w = (float)v[e] + (float)rr[e];
                        if (a.relu) w = w > 0.f ? w : 0.f;
                        v[e] = (bf16)w;
                    }
                }
                *reinterpret_cast<bf16x8*>(a.out + o) = v;
            }
        }
        return;
    }
    if (x >= a.Wo) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ty0 + rg * 4 + i;
        if (y >= a.Ho) continue;
        const long m = ((long)b * a.Ho + y) * a.Wo + x;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + j * 16 + (lane >> 4) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ne = n + e;
                if (ne >= a.N) break;
                float v = acc[i][j][e];
                v += a.bmap ? (float)a.bmap[((long)y * a.Wo + x) * a.N + ne] : (a.bias ? a.bias[ne] : 0.f);
                if (a.resid) v += (float)a.resid[m * a.N + ne];
                if (a.relu) v = v > 0.f ? v : 0.f;
                if (a.out) a.out[m * a.N + ne] = (bf16)v;
                if (a.outf) a.outf[m * a.N + ne] = v;
            }
        }
    }
}

// Forward convolutions only (E_FWD); one 16 x 32 tile per block.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_conv3_dl(GemmArgs a,
                                                                                         unsigned long long* wc) {
    // two separate arrays (not one [2][...] array), so that the compiler can tell the loads
    // into one stage from the reads of the other and does not wait for them before reading
    __shared__ __attribute__((aligned(1024))) unsigned char stage0[DSTAGE];
    __shared__ __attribute__((aligned(1024))) unsigned char stage1[DSTAGE];
    __shared__ __attribute__((aligned(16))) float bias_s[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, rg = wave & 3, cx = wave >> 2;
    const int tiles_x = (a.Wo + DTX - 1) / DTX, tiles_y = (a.Ho + DTY - 1) / DTY;
    int t = blockIdx.x;
    const int tx0 = (t % tiles_x) * DTX;
    t /= tiles_x;
    const int ty0 = (t % tiles_y) * DTY;
    const int b = t / tiles_y;
    const int n0 = blockIdx.y * 64;
    if (a.st && !(a.st[a.rhs0 + b].active && !a.st[a.rhs0 + b].cycdone)) return;
    if (wc && tid == 0) {
        const int my = a.Ho - ty0 < DTY ? a.Ho - ty0 : DTY, mx = a.Wo - tx0 < DTX ? a.Wo - tx0 : DTX;
        const int nr = a.N - n0 < 64 ? a.N - n0 : 64;
        work_atomic(wc, 2ull * my * mx * nr * (unsigned long long)(9 * (a.c1 + a.c2)));
    }
    if (tid < 64) bias_s[tid] = a.bias && n0 + tid < a.N ? a.bias[n0 + tid] : 0.f;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    DlStage ds;
    ds.tile(a, lane, wave, ty0, tx0, 0 >= a.c1);
    ds.wset(a, lane, wave, n0);
    const int nchunk = (a.c1 + a.c2) / HC;
    ds.issue(a, wave, b, 0, stage0);
    // chunk ch is multiplied out of cur while chunk ch + 1 loads into next
    auto step = [&](int ch, unsigned char* next, const unsigned char* cur) {
        __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of chunk ch have landed
        __syncthreads();                 // everyone's have, and nobody still reads the other stage
        if (ch + 1 < nchunk) {
            const int c0 = (ch + 1) * HC;
            if (c0 == a.c1) ds.tile(a, lane, wave, ty0, tx0, 1);
            ds.issue(a, wave, b, c0, next);
        }
        const bf16* P = reinterpret_cast<const bf16*>(cur);
        dl_mma(P, P + DPBYTES / 2, acc, lane, rg, cx);
    };
    for (int ch = 0; ch < nchunk; ch += 2) {
        step(ch, stage1, stage0);
        if (ch + 1 < nchunk) step(ch + 1, stage0, stage1);
    }
    __syncthreads();   // both stages free for the epilogue
    dl_epilogue(a, acc, b, ty0, tx0, n0, tid, reinterpret_cast<bf16*>(stage0), bias_s);
}

// ------------------------------------------------------------------ persistent up-convolution
// Forward 2x2 stride-2 transposed convolution as a GEMM D[M x N] = A[M x K] W^T
// (M input pixels, K = C_in, N = 4 C_out: column n is phase (n / C_out) of output
// channel n % C_out).  The implicit GEMM reloads a block's 128 x K weight slab
// for every 64 pixels, which at these shapes is most of its memory traffic;
// here a block keeps its slab in LDS for the whole launch and walks 64-pixel
// tiles (blockIdx.x, + gridDim.x, ...), the next tile's pixels loaded into
// registers while the current one is multiplied and written out through LDS.
constexpr int UP_BM = 64, UP_BN = 128;
// F32 = true also writes the FP32 copy of the output (the layer tests); kept out of the bf16-only
// form so that its tile loop issues a fixed number of stores.
template <int K, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K <= 64 ? 2 : 1))) void k_upconv(GemmArgs a,
                                                                                                       unsigned long long* wc) {
    constexpr int KP = K + 8;                       // padded LDS row (bf16)
    constexpr int ASEG = UP_BM * K / 8;             // 16-byte segments of a pixel tile
    constexpr int APT = (ASEG + 255) / 256;
    constexpr int OSP = UP_BN + 8;                  // output staging row (bf16)
    __shared__ __attribute__((aligned(16))) bf16 Ws[UP_BN][KP];
    __shared__ __attribute__((aligned(16))) bf16 As[2][UP_BM][KP];
    __shared__ __attribute__((aligned(16))) bf16 Os[UP_BM][OSP];
    __shared__ __attribute__((aligned(16))) float bias_s[UP_BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;        // wave tile: 32 pixels x 64 columns
    const int n0 = blockIdx.y * UP_BN;
    const int cout = a.N >> 2;
    const long ntm = (a.M + UP_BM - 1) / UP_BM;
    // skip tiles of samples whose RHS is inactive (a tile lies in one sample when Ho Wo % 64 == 0)
    const long hw = (long)a.Ho * a.Wo;
    // the samples' RHS flags, read once into LDS: a global load in the tile loop would make the
    // wave wait for all of its outstanding memory operations, the previous tile's stores included
    __shared__ unsigned char live_s[256];
    const bool skip_ok = a.st && hw % UP_BM == 0 && a.B <= 256;
    if (skip_ok)
        for (int i = tid; i < a.B; i += 256) live_s[i] = a.st[a.rhs0 + i].active && !a.st[a.rhs0 + i].cycdone;
    __syncthreads();
    auto live = [&](long mt) { return !skip_ok || live_s[(int)(mt * UP_BM / hw)]; };
    auto next_tile = [&](long mt) {
        while (mt < ntm && !live(mt)) mt += gridDim.x;
        return mt;
    };
    long mt = next_tile(blockIdx.x);
    if (mt >= ntm) return;   // the same decision for every thread of the block
    for (int sg = tid; sg < UP_BN * (K / 8); sg += 256) {
        const int row = sg / (K / 8), sub = sg - row * (K / 8);
        *reinterpret_cast<bf16x8*>(&Ws[row][sub * 8]) =
            n0 + row < a.N ? ld8(a.w + (long)(n0 + row) * a.K + sub * 8) : zero8();
    }
    if (tid < UP_BN) bias_s[tid] = a.bias && n0 + tid < a.N ? a.bias[(n0 + tid) % cout] : 0.f;
    const unsigned arec = (unsigned)((long)a.M * K * 2);
    const __amdgpu_buffer_rsrc_t ra = brsrc(a.a1, arec);   // input pixels [M][K] (one sample after another)
    bf16x8 ra_v[APT];
    auto issue = [&](long t) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const int sg = tid + q * 256;
            const int row = sg / (K / 8), sub = sg - row * (K / 8);
            const long m = t * UP_BM + row;
            ra_v[q] = bload8(ra, sg < ASEG && m < a.M ? (unsigned)((m * K + sub * 8) * 2) : arec);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const int sg = tid + q * 256;
            if (sg < ASEG) {
                const int row = sg / (K / 8), sub = sg - row * (K / 8);
                *reinterpret_cast<bf16x8*>(&As[buf][row][sub * 8]) = ra_v[q];
            }
        }
    };
    const unsigned orec = (unsigned)((long)a.B * 4 * hw * cout * 2);
    const __amdgpu_buffer_rsrc_t ro = brsrc(a.out, orec);
    unsigned long long work = 0;
    issue(mt);
    int buf = 0;
    while (true) {
        store(buf);
        __syncthreads();   // the tile is in As[buf]; the previous tile's output staging has been read
        const long mn = next_tile(mt + gridDim.x);
        if (mn < ntm) issue(mn);
        f32x4 acc[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += 32) {
            bf16x8 fa[2], fb[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                fa[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 32 + i * 16 + (lane & 15)][k0 + (lane >> 4) * 8]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                fb[j] = *reinterpret_cast<const bf16x8*>(&Ws[wn * 64 + j * 16 + (lane & 15)][k0 + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j], fa[i], acc[i][j], 0, 0, 0);
        }
        // acc[i][j][e]: pixel wm*32 + 16 i + l%16, column wn*64 + 16 j + 4 (l/16) + e
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ml = wm * 32 + i * 16 + (lane & 15);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int nl = wn * 64 + j * 16 + (lane >> 4) * 4;
                const float4 bb = *reinterpret_cast<const float4*>(bias_s + nl);
                f32x4 v = acc[i][j];
                v[0] += bb.x;
                v[1] += bb.y;
                v[2] += bb.z;
                v[3] += bb.w;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = a.relu && v[e] < 0.f ? 0.f : v[e];
                bf16x4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
                *reinterpret_cast<bf16x4*>(&Os[ml][nl]) = o;
                const long m = mt * UP_BM + ml;
                const int n = n0 + nl;
                if (F32 && m < a.M && n < a.N) {
                    const Pix p = pix_of(m, a.Ho, a.Wo);
                    const int ad = n / cout, co = n - ad * cout;
                    *reinterpret_cast<f32x4*>(
                        a.outf + (((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) * cout + co) = v;
                }
            }
        }
        __syncthreads();
        // 64 pixels x 128 columns in 16-byte groups, four per thread, always issued (groups past
        // M or N get an offset past the end of the output, which the range check drops)
#pragma unroll
        for (int r = 0; r < UP_BM * UP_BN / 8 / 256; ++r) {
            const int k = tid + r * 256;
            const int ml = k / (UP_BN / 8), c = k - ml * (UP_BN / 8);
            const long m = mt * UP_BM + ml;
            const int n = n0 + c * 8;
            unsigned off = orec;
            if (m < a.M && n < a.N) {
                const Pix p = pix_of(m, a.Ho, a.Wo);
                const int ad = n / cout, co = n - ad * cout;
                off = (unsigned)(((((long)p.b * 2 * a.Ho + 2 * p.y + (ad >> 1)) * (2 * a.Wo) + 2 * p.x + (ad & 1)) * cout + co) * 2);
            }
            __builtin_amdgcn_raw_buffer_store_b128(
                __builtin_bit_cast(u32x4s, *reinterpret_cast<const bf16x8*>(&Os[ml][c * 8])), ro, off, 0, 0);
        }
        if (wc) {
            const long mr = a.M - mt * UP_BM < UP_BM ? a.M - mt * UP_BM : UP_BM;
            const int nr = a.N - n0 < UP_BN ? a.N - n0 : UP_BN;
            work += 2ull * (unsigned long long)mr * nr * K;
        }
        if (mn >= ntm) break;
        mt = mn;
        buf ^= 1;
    }
    if (wc && tid == 0) work_atomic(wc, work);
}

// Persistent form for layers of NCH * 32 input channels (NCH = 1, 2) and at most
// BN output channels: the block loads all its weights into LDS once, walks over
// (tile, chunk) items with a stride of gridDim.x tiles, and prefetches the next
// item's patch into registers while the current one runs.
template <int BN, int FLIP, int EPI, int NCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NCH == 1 ? 3 : 2))) void k_conv3_pers(GemmArgs a, unsigned long long* wc) {
    constexpr int WTN = BN / 16;
    constexpr int WLD = NCH * HC + 8;
    __shared__ __attribute__((aligned(16))) bf16 Ps[HP * HP][HLD];
    __shared__ __attribute__((aligned(16))) bf16 Ws[9][BN][WLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (a.Wo + HT - 1) / HT, tiles_y = (a.Ho + HT - 1) / HT;
    const int tps = tiles_x * tiles_y;
    const int ntiles = a.B * tps;
    const int n0 = blockIdx.y * BN;
    // the samples' RHS flags, read once into LDS: a global load in the tile loop would make the
    // wave wait for all of its outstanding memory operations, the previous tile's stores included
    __shared__ unsigned char live_s[256];
    const bool flags_lds = a.st && a.B <= 256;
    if (flags_lds)
        for (int i = tid; i < a.B; i += 256) live_s[i] = a.st[a.rhs0 + i].active && !a.st[a.rhs0 + i].cycdone;
    __syncthreads();
    auto next_tile = [&](int t) {
        while (t < ntiles && a.st &&
               !(flags_lds ? live_s[t / tps] : a.st[a.rhs0 + t / tps].active && !a.st[a.rhs0 + t / tps].cycdone))
            t += gridDim.x;
        return t;
    };
    int t = next_tile(blockIdx.x);
    if (t >= ntiles) return;   // the same decision for every thread of the block
    __shared__ __attribute__((aligned(16))) float bias_s[BN];
    if (EPI == E_FWD && tid < BN) bias_s[tid] = a.bias && n0 + tid < a.N ? a.bias[n0 + tid] : 0.f;
    // all weights of the block's output channels, once
    constexpr int C = NCH * HC;
    for (int sg = tid; sg < 9 * BN * (C / 8); sg += 256) {
        const int row = sg / (C / 8), sub = sg - row * (C / 8);   // row = tap * BN + n
        const int tap = row / BN, n = row - tap * BN;
        *reinterpret_cast<bf16x8*>(&Ws[tap][n][sub * 8]) =
            n0 + n < a.N ? ld8(a.w + (long)(n0 + n) * a.K + tap * C + sub * 8) : zero8();
    }
    HaloStage<BN> st;
    st.load(a, tid, t / tps, ((t / tiles_x) % tiles_y) * HT, (t % tiles_x) * HT, n0, 0, false);
    int ch = 0;
    unsigned long long work = 0;   // algorithmic flops of this block, one counter update at the end
    f32x4 acc[4][WTN];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    while (true) {
        st.store(Ps, Ws, tid, false);
        __syncthreads();
        int tn = t, chn = ch + 1;
        if (chn == NCH) {
            chn = 0;
            tn = next_tile(t + gridDim.x);
        }
        if (tn < ntiles)
            st.load(a, tid, tn / tps, ((tn / tiles_x) % tiles_y) * HT, (tn % tiles_x) * HT, n0, chn * HC, false);
        halo_mma<BN, FLIP, WLD>(Ps, Ws, ch * HC, acc, lane, wave);
        __syncthreads();
        if (ch == NCH - 1) {
            const int b = t / tps, ty0 = ((t / tiles_x) % tiles_y) * HT, tx0 = (t % tiles_x) * HT;
            work += halo_work(a, ty0, tx0, n0, BN);
            constexpr bool fits = sizeof(Ps) >= 256 * (BN + 8) * sizeof(bf16);
            if (EPI == E_FWD && fits && halo_lds_epilogue_ok<BN>(a))
                halo_epilogue_lds<BN>(a, acc, b, ty0, tx0, n0, tid, &Ps[0][0], bias_s);
            else
                halo_epilogue<BN, EPI>(a, acc, b, ty0, tx0, n0, lane, wave);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < WTN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
        if (tn >= ntiles) break;
        t = tn;
        ch = chn;
    }
    if (wc && tid == 0) work_atomic(wc, work);
}

// ------------------------------------------------------------------ first layer (few input channels)
// 3x3 stride-1 convolution with C <= 4 input channels and N <= 64 outputs (the
// networks' first layers, C = 2): FP32 FMAs with the weights in LDS.  Thread t
// of a block computes output channels 8 (t % (N/8)) .. +7 of one pixel, so the
// lanes of a wave write consecutive 16-byte pieces of the NHWC output.  The
// implicit GEMM would pad K = 9 C up to 32 and gather element by element.
constexpr int SC_MAXK = 36, SC_MAXN = 64;
template <int C>
__global__ __launch_bounds__(256) void k_conv3_smallc(GemmArgs a, unsigned long long* wc) {
    __shared__ float Wl[SC_MAXK][SC_MAXN];
    __shared__ float bl[SC_MAXN];
    constexpr int K9 = 9 * C;
    const int N = a.N, G = N / 8;              // 8-channel groups per pixel
    for (int i = threadIdx.x; i < K9 * N; i += 256) {
        const int k = i / N, n = i - k * N;
        Wl[k][n] = (float)a.w[(long)n * a.K + k];
    }
    for (int n = threadIdx.x; n < N; n += 256) bl[n] = a.bias[n];
    __syncthreads();
    const long nq = a.M * G;
    if (wc && threadIdx.x == 0) {
        unsigned long long cnt = 0;
        for (long q0 = (long)blockIdx.x * 256; q0 < nq; q0 += (long)gridDim.x * 256)
            cnt += (unsigned long long)(nq - q0 < 256 ? nq - q0 : 256);
        work_atomic(wc, 2ull * cnt * 8 * K9);
    }
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < nq; q += (long)gridDim.x * 256) {
        const long m = (long)((unsigned)q / (unsigned)G);
        const int n8 = (int)((unsigned)q - (unsigned)m * (unsigned)G) * 8;
        const Pix p = pix_of(m, a.Ho, a.Wo);
        if (a.st && !(a.st[a.rhs0 + p.b].active && !a.st[a.rhs0 + p.b].cycdone)) continue;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = bl[n8 + e];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int yi = p.y + tap / 3 - 1, xi = p.x + tap % 3 - 1;
            if (yi < 0 || yi >= a.Hi || xi < 0 || xi >= a.Wi) continue;
            const bf16* src = a.a1 + p.b * a.abs1 + ((long)yi * a.Wi + xi) * C;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float x = (float)src[c];
                const float4 w0 = *reinterpret_cast<const float4*>(&Wl[tap * C + c][n8]);
                const float4 w1 = *reinterpret_cast<const float4*>(&Wl[tap * C + c][n8 + 4]);
                v[0] += x * w0.x;
                v[1] += x * w0.y;
                v[2] += x * w0.z;
                v[3] += x * w0.w;
                v[4] += x * w1.x;
                v[5] += x * w1.y;
                v[6] += x * w1.z;
                v[7] += x * w1.w;
            }
        }
        if (a.resid) {
            const bf16x8 r = *reinterpret_cast<const bf16x8*>(a.resid + m * N + n8);
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] += (float)r[e];
        }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (a.relu) v[e] = v[e] > 0.f ? v[e] : 0.f;
            o[e] = (bf16)v[e];
        }
        *reinterpret_cast<bf16x8*>(a.out + m * N + n8) = o;
        if (a.outf) {
            *reinterpret_cast<f32x4*>(a.outf + m * N + n8) = (f32x4){v[0], v[1], v[2], v[3]};
            *reinterpret_cast<f32x4*>(a.outf + m * N + n8 + 4) = (f32x4){v[4], v[5], v[6], v[7]};
        }
    }
}

// Two-channel first layer on the matrix cores: K = 9 taps x 2 channels = 18,
// padded to one 32-deep MFMA step.  Lane l gathers, for pixel l%16 of a
// 16-pixel row segment, the 8 (tap, channel) values k = 8(l/16) .. +7 with
// 4-byte loads; the weight fragments stay in registers for the whole launch.
// Waves walk over row segments with a grid stride.
template <int NT>
__global__ __launch_bounds__(256) void k_conv3_first2(GemmArgs a, unsigned long long* wc) {
    const int lane = threadIdx.x & 63;
    const long wave0 = ((long)blockIdx.x * 256 + threadIdx.x) >> 6;
    const long nwaves = (long)gridDim.x * 4;
    const int segs_x = (a.Wo + 15) / 16;
    const long nseg = (long)a.B * a.Ho * segs_x;
    const int kg = lane >> 4;                  // k = 8 kg .. 8 kg + 7
    bf16x8 fw[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) fw[j] = ld8(a.w + (long)(j * 16 + (lane & 15)) * a.K + kg * 8);
    float bias[NT][4];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[j][e] = a.bias[j * 16 + kg * 4 + e];
    // per-wave LDS rows for whole-line stores: N = 16 NT channels per pixel, padded
    constexpr int FSP = NT * 16 + 8;
    __shared__ __attribute__((aligned(16))) bf16 fl[4][16 * FSP];
    bf16* wl = fl[threadIdx.x >> 6];
    const bool staged = a.out && !a.outf && !a.resid && a.N == NT * 16;
    unsigned long long work = 0;
    for (long sgi = wave0; sgi < nseg; sgi += nwaves) {
        const int sx = (int)(sgi % segs_x);
        const long rowi = sgi / segs_x;
        const int y = (int)(rowi % a.Ho), b = (int)(rowi / a.Ho);
        if (a.st && !(a.st[a.rhs0 + b].active && !a.st[a.rhs0 + b].cycdone)) continue;
        const int x = sx * 16 + (lane & 15);
        // gather taps 4 kg .. 4 kg + 3 (two channels each); taps >= 9 are the zero padding
        bf16x8 fx = zero8();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int tap = kg * 4 + q;
            if (tap >= 9) break;
            const int yi = y + tap / 3 - 1, xi = x + tap % 3 - 1;
            if (x < a.Wo && yi >= 0 && yi < a.Hi && xi >= 0 && xi < a.Wi) {
                // both channels of the tap in one 4-byte load
                const bf16* src = a.a1 + b * a.abs1 + ((long)yi * a.Wi + xi) * 2;
                const bf16x2g v2 = *reinterpret_cast<const bf16x2g*>(src);
                fx[2 * q] = v2[0];
                fx[2 * q + 1] = v2[1];
            }
        }
        if (x < a.Wo) work += 2ull * 18 * a.N;
        const long m = ((long)b * a.Ho + y) * a.Wo + x;
        if (staged) {
            // the segment's 16 pixels x N channels are contiguous in memory: finish them
            // into the wave's LDS rows and store 16 contiguous bytes per lane
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const f32x4 acc =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fx, (f32x4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                bf16x4g o;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[e] + bias[j][e];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    o[e] = (bf16)v;
                }
                *reinterpret_cast<bf16x4g*>(wl + (lane & 15) * FSP + j * 16 + kg * 4) = o;
            }
            __builtin_amdgcn_wave_barrier();
            const long m0 = ((long)b * a.Ho + y) * a.Wo + sx * 16;
            for (int k = lane; k < 16 * (NT * 2); k += 64) {
                const int px = k / (NT * 2), c = k - px * (NT * 2);
                if (sx * 16 + px < a.Wo)
                    *reinterpret_cast<bf16x8*>(a.out + (m0 + px) * a.N + c * 8) =
                        *reinterpret_cast<const bf16x8*>(wl + px * FSP + c * 8);
            }
            __builtin_amdgcn_wave_barrier();
            continue;
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fx, (f32x4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            if (x >= a.Wo) continue;
            const int n = j * 16 + kg * 4;
            bf16x4g o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = acc[e] + bias[j][e];
                if (a.resid) v += (float)a.resid[m * a.N + n + e];
                if (a.relu) v = v > 0.f ? v : 0.f;
                o[e] = (bf16)v;
                acc[e] = v;
            }
            if (a.out) *reinterpret_cast<bf16x4g*>(a.out + m * a.N + n) = o;
            if (a.outf) *reinterpret_cast<f32x4*>(a.outf + m * a.N + n) = acc;
        }
    }
    if (wc) {
        // one counter update per wave
        unsigned long long tot = work;
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
        if (lane == 0) work_atomic(wc, tot);
    }
}

static bool first2_ok(const GemmArgs& a) {
    return a.gmode == G_CONV && a.stride == 1 && a.epi == E_FWD && !a.bmap && a.c2 == 0 && a.c1 == 2 &&
           a.N % 16 == 0 && a.N <= 64 && a.K >= 32;
}

static bool smallc_ok(const GemmArgs& a) {
    return a.gmode == G_CONV && a.stride == 1 && a.epi == E_FWD && !a.bmap && a.c2 == 0 && a.c1 >= 1 && a.c1 <= 4 &&
           a.N % 8 == 0 && a.N <= SC_MAXN && a.K >= 9 * a.c1;
}

// Resident blocks of a kernel on the whole device (cached per kernel).
template <typename K>
static int resident_blocks(K kernel, int& cache) {
    if (cache > 0) return cache;
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu <= 0)
        return 256;
    cache = per_cu * cus;
    return cache;
}

// ------------------------------------------------------------------ fused 32-channel residual block
// y = x + W2 * ReLU(W1 * x + b1) + b2 for 32 channels (the networks' first
// level, where the convolutions are bound by HBM traffic).  A block keeps both
// weight sets in LDS and walks over 14 x 14 output tiles: it stages the 18 x 18
// input patch, computes h = ReLU(W1 * x + b1) on the surrounding 16 x 16 grid
// (zero outside the image, the padding of the second convolution), writes h
// back into the patch buffer with a zero border, and runs the second
// convolution there; the residual is read from the staged input.  The
// intermediate h never reaches HBM.
constexpr int RT = HT - 2;   // output tile edge (14)

__global__ __launch_bounds__(256) void k_resblock32(ResArgs a, unsigned long long* wc) {
    __shared__ __attribute__((aligned(16))) bf16 Ps[HP * HP][HLD];
    __shared__ __attribute__((aligned(16))) bf16 W1s[9][32][HLD];
    __shared__ __attribute__((aligned(16))) bf16 W2s[9][32][HLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (a.W + RT - 1) / RT, tiles_y = (a.H + RT - 1) / RT, tps = tiles_x * tiles_y;
    const int ntiles = a.B * tps;
    // the samples' RHS flags, read once into LDS: a global load in the tile loop would make the
    // wave wait for all of its outstanding memory operations, the previous tile's stores included
    __shared__ unsigned char live_s[256];
    const bool flags_lds = a.st && a.B <= 256;
    if (flags_lds)
        for (int i = tid; i < a.B; i += 256) live_s[i] = a.st[a.rhs0 + i].active && !a.st[a.rhs0 + i].cycdone;
    __syncthreads();
    auto next_tile = [&](int t) {
        while (t < ntiles && a.st &&
               !(flags_lds ? live_s[t / tps] : a.st[a.rhs0 + t / tps].active && !a.st[a.rhs0 + t / tps].cycdone))
            t += gridDim.x;
        return t;
    };
    int t = next_tile(blockIdx.x);
    if (t >= ntiles) return;   // the same decision for every thread of the block
    __shared__ float bl[2][32];   // both layers' biases, read from LDS in every tile's epilogues
    if (tid < 64) bl[tid >> 5][tid & 31] = (tid < 32 ? a.b1 : a.b2)[tid & 31];
    for (int sg = tid; sg < 9 * 32 * 4; sg += 256) {
        const int row = sg >> 2, sub = sg & 3, tap = row >> 5, n = row & 31;
        *reinterpret_cast<bf16x8*>(&W1s[tap][n][sub * 8]) = ld8(a.w1 + (long)n * a.K1 + tap * 32 + sub * 8);
        *reinterpret_cast<bf16x8*>(&W2s[tap][n][sub * 8]) = ld8(a.w2 + (long)n * a.K2 + tap * 32 + sub * 8);
    }
    // the input patch of a tile with output origin (oy0, ox0) starts at (oy0 - 2, ox0 - 2);
    // HaloStage loads the patch of a 16 x 16 grid at origin (ty0, tx0) from (ty0 - 1, tx0 - 1)
    GemmArgs g{};
    g.a1 = a.x;
    g.c1 = 32;
    g.abs1 = (long)a.H * a.W * 32;
    g.Hi = a.H;
    g.Wi = a.W;
    HaloStage<32> st;
    auto origin = [&](int tt, int& b, int& oy0, int& ox0) {
        b = tt / tps;
        oy0 = ((tt / tiles_x) % tiles_y) * RT;
        ox0 = (tt % tiles_x) * RT;
    };
    int b, oy0, ox0;
    origin(t, b, oy0, ox0);
    st.load(g, tid, b, oy0 - 1, ox0 - 1, 0, 0, false);
    unsigned long long work = 0;
    typedef __bf16 bf16x4r __attribute__((ext_vector_type(4)));
    while (true) {
        origin(t, b, oy0, ox0);
        st.store(Ps, W1s, tid, false);
        __syncthreads();
        const int tn = next_tile(t + gridDim.x);
        if (tn < ntiles) {
            int bn, yn, xn;
            origin(tn, bn, yn, xn);
            st.load(g, tid, bn, yn - 1, xn - 1, 0, 0, false);
        }
        // stage A: h on the 16 x 16 grid at image origin (oy0 - 1, ox0 - 1)
        f32x4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
        halo_mma<32, 0>(Ps, W1s, 0, acc, lane, wave);
        // residual x at the same grid positions (patch offset +1) before the patch is overwritten
        const int px = lane & 15;
        bf16x4r res[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                res[i][j] = *reinterpret_cast<const bf16x4r*>(
                    &Ps[(wave * 4 + i + 1) * HP + px + 1][j * 16 + (lane >> 4) * 4]);
        __syncthreads();
        // h (ReLU, zero outside the image) into the patch buffer at offset +1, zero border
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int py = wave * 4 + i;
            const int yi = oy0 - 1 + py, xi = ox0 - 1 + px;
            const bool in = yi >= 0 && yi < a.H && xi >= 0 && xi < a.W;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = j * 16 + (lane >> 4) * 4;
                bf16x4r hv;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = acc[i][j][e] + bl[0][n + e];
                    hv[e] = (bf16)(in && v > 0.f ? v : 0.f);
                }
                *reinterpret_cast<bf16x4r*>(&Ps[(py + 1) * HP + px + 1][n]) = hv;
            }
        }
        for (int q = tid; q < (4 * HP - 4) * 4; q += 256) {   // the 68 border pixels x 4 segments
            const int bp = q >> 2, sub = q & 3;
            int pyb, pxb;
            if (bp < HP) {
                pyb = 0;
                pxb = bp;
            } else if (bp < 2 * HP) {
                pyb = HP - 1;
                pxb = bp - HP;
            } else {
                const int r = bp - 2 * HP;   // 0 .. 2*(HP-2)-1
                pyb = 1 + (r >> 1);
                pxb = (r & 1) ? HP - 1 : 0;
            }
            *reinterpret_cast<bf16x8*>(&Ps[pyb * HP + pxb][sub * 8]) = zero8();
        }
        __syncthreads();
        // stage B: second convolution over h; grid positions 1 .. 14 are the outputs
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
        halo_mma<32, 0>(Ps, W2s, 0, acc, lane, wave);
        // the RT x RT outputs go through the patch buffer so that every pixel's 64 bytes
        // leave in one store instruction (16 contiguous bytes per lane)
        __syncthreads();
        bf16* ob = &Ps[0][0];
        constexpr int OSP = 40;   // bf16 per output pixel in LDS
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int py = wave * 4 + i;
            if (py < 1 || py > RT || px < 1 || px > RT) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = j * 16 + (lane >> 4) * 4;
                bf16x4r o;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (bf16)(acc[i][j][e] + bl[1][n + e] + (float)res[i][j][e]);
                *reinterpret_cast<bf16x4r*>(ob + ((py - 1) * RT + px - 1) * OSP + n) = o;
            }
        }
        __syncthreads();
        // a fixed number of stores per thread (pixels outside the image or past the tile are
        // written past the end of the buffer, which the buffer's range check drops), so that
        // the wait for the next tile's prefetched patch need not also wait for these stores
        {
            const unsigned nrec = (unsigned)((long)a.B * a.H * a.W * 32 * 2);
            const __amdgpu_buffer_rsrc_t ro = brsrc(a.out, nrec);
#pragma unroll
            for (int r = 0; r < (RT * RT * 4 + 255) / 256; ++r) {
                const int k = tid + r * 256;
                const int p = k >> 2, c = k & 3;
                const int y = oy0 + p / RT, x = ox0 + p % RT;
                const bool ok = k < RT * RT * 4 && y < a.H && x < a.W;
                const unsigned off = ok ? (unsigned)(((((long)b * a.H + y) * a.W + x) * 32 + c * 8) * 2) : nrec;
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(ob + (ok ? p : 0) * OSP + c * 8);
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4s, v), ro, off, 0, 0);
            }
        }
        if (wc) {
            const int my = a.H - oy0 < RT ? a.H - oy0 : RT, mx = a.W - ox0 < RT ? a.W - ox0 : RT;
            work += 2ull * 2ull * my * mx * 32ull * 288ull;   // both convolutions, valid outputs only
        }
        __syncthreads();
        if (tn >= ntiles) break;
        t = tn;
    }
    if (wc && tid == 0) work_atomic(wc, work);
}

// Solver first layer + level-0 context convolution in one persistent kernel.
// Per 16 x 16 output tile: the 20 x 20 two-channel input patch goes to LDS, the
// 18 x 18 h0 patch is computed from it with one 32-deep MFMA step per 16 pixels
// (first layer weights in registers, taps 9..15 of the K step zero) and written
// to the patch buffer (zero outside the image: the context convolution's
// padding), then the context convolution runs on it as in the halo kernels.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_first_ctx(FirstCtxArgs a,
                                                                                         unsigned long long* wc) {
    constexpr int RP = HT + 4;   // input patch edge
    __shared__ __attribute__((aligned(16))) bf16 Ps[HP * HP][HLD];
    __shared__ __attribute__((aligned(16))) bf16 Ws[9][32][HLD];
    __shared__ unsigned Rs[RP * RP];   // two bf16 channels per pixel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (a.W + HT - 1) / HT, tiles_y = (a.H + HT - 1) / HT, tps = tiles_x * tiles_y;
    const int ntiles = a.B * tps;
    // the samples' RHS flags, read once into LDS (see k_conv3_pers)
    __shared__ unsigned char live_s[256];
    const bool flags_lds = a.st && a.B <= 256;
    if (flags_lds)
        for (int i = tid; i < a.B; i += 256) live_s[i] = a.st[a.rhs0 + i].active && !a.st[a.rhs0 + i].cycdone;
    __syncthreads();
    auto next_tile = [&](int t) {
        while (t < ntiles && a.st &&
               !(flags_lds ? live_s[t / tps] : a.st[a.rhs0 + t / tps].active && !a.st[a.rhs0 + t / tps].cycdone))
            t += gridDim.x;
        return t;
    };
    int t = next_tile(blockIdx.x);
    if (t >= ntiles) return;   // the same decision for every thread of the block
    for (int sg = tid; sg < 9 * 32 * 4; sg += 256) {
        const int row = sg >> 2, sub = sg & 3, tap = row >> 5, n = row & 31;
        *reinterpret_cast<bf16x8*>(&Ws[tap][n][sub * 8]) = ld8(a.wh + (long)n * a.Kh + tap * 32 + sub * 8);
    }
    const int kg = lane >> 4;   // this lane's k = 8 kg .. 8 kg + 7: taps 4 kg .. 4 kg + 3, two channels each
    bf16x8 fw[2];
    float b0v[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        fw[j] = ld8(a.w0 + (long)(j * 16 + (lane & 15)) * a.K0 + kg * 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) b0v[j][e] = a.b0[j * 16 + kg * 4 + e];
    }
    auto origin = [&](int tt, int& b, int& ty0, int& tx0) {
        b = tt / tps;
        ty0 = ((tt / tiles_x) % tiles_y) * HT;
        tx0 = (tt % tiles_x) * HT;
    };
    unsigned rr[2];
    // two 4-byte loads per thread and tile, always issued (pixels outside the image or the patch
    // read past the end of the input and get zeros), so that their count is fixed
    const unsigned rrec = (unsigned)((long)a.B * a.H * a.W * 2 * 2);
    const __amdgpu_buffer_rsrc_t rsr = brsrc(a.r, rrec);
    auto rload = [&](int tt) {
        int b, ty0, tx0;
        origin(tt, b, ty0, tx0);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int idx = tid + q * 256;
            const int py = idx / RP, px = idx - py * RP;
            const int yi = ty0 - 2 + py, xi = tx0 - 2 + px;
            const bool in = idx < RP * RP && yi >= 0 && yi < a.H && xi >= 0 && xi < a.W;
            rr[q] = __builtin_amdgcn_raw_buffer_load_b32(rsr, in ? (unsigned)((((long)b * a.H + yi) * a.W + xi) * 4) : rrec,
                                                         0, 0);
        }
    };
    GemmArgs g{};   // the epilogue's view of the output
    g.B = a.B;
    g.Ho = a.H;
    g.Wo = a.W;
    g.N = 32;
    g.bmap = a.bmap;
    g.relu = 1;
    g.out = a.out;
    rload(t);
    unsigned long long work = 0;
    typedef __bf16 bf16x2f __attribute__((ext_vector_type(2)));
    while (true) {
        int b, ty0, tx0;
        origin(t, b, ty0, tx0);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (tid + q * 256 < RP * RP) Rs[tid + q * 256] = rr[q];
        __syncthreads();
        const int tn = next_tile(t + gridDim.x);
        if (tn < ntiles) rload(tn);
        // h0 on the 18 x 18 patch at image origin (ty0 - 1, tx0 - 1), 16 pixels per MFMA step
        for (int grp = wave; grp < (HP * HP + 15) / 16; grp += 4) {
            const int p = grp * 16 + (lane & 15);
            const int pc = p < HP * HP ? p : HP * HP - 1;
            const int py = pc / HP, px = pc - py * HP;
            bf16x8 fx = zero8();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int tap = kg * 4 + q;
                if (tap >= 9) break;
                const bf16x2f v2 = __builtin_bit_cast(bf16x2f, Rs[(py + tap / 3) * RP + px + tap % 3]);
                fx[2 * q] = v2[0];
                fx[2 * q + 1] = v2[1];
            }
            const int yi = ty0 - 1 + py, xi = tx0 - 1 + px;
            const bool in = p < HP * HP && yi >= 0 && yi < a.H && xi >= 0 && xi < a.W;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fx, (f32x4){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                bf16x4 o;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = acc[e] + b0v[j][e];
                    o[e] = (bf16)(in && v > 0.f ? v : 0.f);
                }
                if (p < HP * HP) *reinterpret_cast<bf16x4*>(&Ps[p][j * 16 + kg * 4]) = o;
            }
        }
        __syncthreads();
        f32x4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
        halo_mma<32, 0>(Ps, Ws, 0, acc, lane, wave);
        __syncthreads();
        if (wc) {
            const int my = a.H - ty0 < HT ? a.H - ty0 : HT, mx = a.W - tx0 < HT ? a.W - tx0 : HT;
            work += (unsigned long long)my * mx * (2ull * 18 * 32 + 2ull * 288 * 32);
        }
        halo_epilogue_lds<32>(g, acc, b, ty0, tx0, 0, tid, &Ps[0][0], nullptr);
        if (tn >= ntiles) break;
        t = tn;
    }
    if (wc && tid == 0) work_atomic(wc, work);
}

int launch_first_ctx(const FirstCtxArgs& a, hipStream_t s) {
    if (a.B <= 0 || a.H <= 0 || a.W <= 0) return HELM_OK;
    if (a.K0 < 32 || a.Kh < 288) return fail(HELM_EINVAL, "first_ctx: weight depths %d, %d below 32, 288", a.K0, a.Kh);
    if ((long)a.B * a.H * a.W >= (1L << 31) / 32) return fail(HELM_EINVAL, "first_ctx: grid too large");
    static int res = 0;
    const int tiles = ((a.H + HT - 1) / HT) * ((a.W + HT - 1) / HT) * a.B;
    const int gx = std::max(1, std::min(tiles, resident_blocks(k_first_ctx, res)));
    TIMED_LAUNCH("k_conv", s, k_first_ctx, dim3(gx), dim3(256), 0, s, a, WORK_COUNTER("k_conv", s));
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

int launch_resblock32(const ResArgs& a, hipStream_t s) {
    if (a.B <= 0 || a.H <= 0 || a.W <= 0) return HELM_OK;
    if (a.K1 < 288 || a.K2 < 288) return fail(HELM_EINVAL, "resblock32: weight depth below 9 x 32");
    if ((long)a.B * a.H * a.W >= (1L << 31) / 32) return fail(HELM_EINVAL, "resblock32: grid too large");
    static int res = 0;
    const int tiles = ((a.H + RT - 1) / RT) * ((a.W + RT - 1) / RT) * a.B;
    const int gx = std::max(1, std::min(tiles, resident_blocks(k_resblock32, res)));
    TIMED_LAUNCH("k_conv", s, k_resblock32, dim3(gx), dim3(256), 0, s, a, WORK_COUNTER("k_conv", s));
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

// The halo kernels apply when every source has a multiple of 32 channels.
static bool halo_ok(const GemmArgs& a) {
    if (!(a.gmode == G_CONV || a.gmode == G_CONVT) || a.stride != 1) return false;
    if (a.c1 % HC || a.c2 % HC) return false;
    if (a.gmode == G_CONV && a.epi != E_FWD) return false;
    if (a.gmode == G_CONVT && a.epi != E_ACC) return false;
    // the staging addresses one sample's input half and the weights with 32-bit byte offsets
    if ((long)a.Hi * a.Wi * std::max(a.c1, a.c2) * 2 + 4096 >= (1L << 31)) return false;
    if ((long)a.N * a.K * 2 >= (1L << 31)) return false;
    // and the epilogue addresses the output (and a residual) with 32-bit byte offsets
    if ((long)a.B * a.Ho * a.Wo * a.N * 2 >= (1L << 31)) return false;
    return a.K >= 9 * (a.c1 + a.c2);
}


template <int BN, int FLIP, int EPI, int NCH>
static void launch_pers(const GemmArgs& a, hipStream_t s, unsigned long long* wc) {
    static int res = 0;
    const int ntiles = ((a.Ho + HT - 1) / HT) * ((a.Wo + HT - 1) / HT) * a.B;
    const int ny = (a.N + BN - 1) / BN;
    const int slots = resident_blocks(k_conv3_pers<BN, FLIP, EPI, NCH>, res);
    const int gx = std::max(1, std::min(ntiles, slots / ny));
    TIMED_LAUNCH("k_conv", s, (k_conv3_pers<BN, FLIP, EPI, NCH>), dim3(gx, ny), dim3(256), 0, s, a, wc);
}

template <int BN, int FLIP, int EPI>
static void launch_single(const GemmArgs& a, hipStream_t s, unsigned long long* wc) {
    const int ntiles = ((a.Ho + HT - 1) / HT) * ((a.Wo + HT - 1) / HT) * a.B;
    TIMED_LAUNCH("k_conv", s, (k_conv3_halo<BN, FLIP, EPI>), dim3(ntiles, (a.N + BN - 1) / BN), dim3(256), 0, s, a,
                 wc);
}

template <int GM, int BM, int BN, int WGM, int WGN>
static void launch_gemm_tile(const GemmArgs& a, hipStream_t s, unsigned long long* wc) {
    dim3 grid((unsigned)((a.M + BM - 1) / BM), (a.N + BN - 1) / BN);
    TIMED_LAUNCH("k_conv", s, (k_gemm<GM, BM, BN, WGM, WGN>), grid, dim3(256), 0, s, a, wc);
}

template <int GM>
// Block tiles: 0: 64 x 64, 1: 128 x 32, 2: 64 x 128, 3: 128 x 64 (pixels x output columns).
static void launch_gemm_pick(const GemmArgs& a, hipStream_t s, unsigned long long* wc, int shape) {
    switch (shape) {
        case 1: launch_gemm_tile<GM, 128, 32, 4, 1>(a, s, wc); break;
        case 2: launch_gemm_tile<GM, 64, 128, 2, 2>(a, s, wc); break;
        case 3: launch_gemm_tile<GM, 128, 64, 2, 2>(a, s, wc); break;
        default: launch_gemm_tile<GM, 64, 64, 2, 2>(a, s, wc); break;
    }
}

// ------------------------------------------------------------------ kernel choice and autotuning
// Every convolution launch picks one of these kernels.  A built-in rule gives
// the default; with autotuning on, the first eager launch of each problem shape
// (outside stream capture) times every applicable candidate on the caller's
// buffers and keeps the fastest for that shape.  Only overwriting epilogues are
// tuned (accumulating ones would add each candidate's result).
enum ConvKernel {
    CK_PERS = 0, CK_HALO32, CK_HALO64, CK_GEMM64, CK_GEMM128, CK_SMALLC, CK_FIRST2, CK_GEMM64W, CK_GEMM128W,
    CK_PERS16, CK_DL64, CK_UPP, CK_GPF64, CK_GPF128, CK_COUNT
};

// The deeper-prefetch implicit GEMM: forward 3 x 3 convolutions writing bf16 (and optionally
// an FP32 copy), sources of a multiple of 32 channels (so K = 9 C, a multiple of GPF_D
// chunks), 32-bit byte offsets.
static bool gemm_pf_ok(const GemmArgs& a) {
    if (a.gmode != G_CONV || a.epi != E_FWD || !a.out || (a.N & 7) != 0) return false;
    if (a.c1 <= 0 || (a.c1 & 31) != 0 || (a.c2 & 31) != 0) return false;
    const int C = a.c1 + a.c2;
    if (a.K != 9 * C || a.kvalid != a.K || (a.K / KC) % GPF_D != 0) return false;
    const long s1 = a.abs1 ? (long)a.B * a.abs1 : (long)a.Hi * a.Wi * a.c1;
    const long s2 = a.abs2 ? (long)a.B * a.abs2 : (long)a.Hi * a.Wi * a.c2;
    return s1 * 2 < (1L << 31) && s2 * 2 < (1L << 31) && (long)a.N * a.K * 2 < (1L << 31) &&
           a.M < (1L << 31);
}

// The persistent up-convolution: K = C_in of 64, 128 or 256, contiguous input, C_out a multiple
// of 8, 32-bit byte offsets.
static bool upconv_ok(const GemmArgs& a) {
    if (a.gmode != G_UP || a.epi != E_UPFWD || !a.out || a.c2 != 0 || a.resid || a.bmap) return false;
    if (!(a.K == a.c1 && (a.c1 == 64 || a.c1 == 128 || a.c1 == 256))) return false;
    if (a.abs1 != (long)a.Hi * a.Wi * a.c1 || a.Ho != a.Hi || a.Wo != a.Wi || (a.N & 31) != 0) return false;
    return (long)a.M * a.K * 2 < (1L << 31) && (long)a.M * a.N * 2 < (1L << 31);
}

template <int K>
static void launch_upconv_k(const GemmArgs& a, hipStream_t s, unsigned long long* wc) {
    static int res = 0;
    const long ntm = (a.M + UP_BM - 1) / UP_BM;
    const int ny = (a.N + UP_BN - 1) / UP_BN;
    const int slots = resident_blocks(k_upconv<K, false>, res);
    const int gx = (int)std::max<long>(1, std::min<long>(ntm, std::max(1, slots / ny)));
    if (a.outf)
        TIMED_LAUNCH("k_conv", s, (k_upconv<K, true>), dim3(gx, ny), dim3(256), 0, s, a, wc);
    else
        TIMED_LAUNCH("k_conv", s, (k_upconv<K, false>), dim3(gx, ny), dim3(256), 0, s, a, wc);
}

static bool ck_applicable(const GemmArgs& a, int ck) {
    const bool halo = halo_ok(a);
    const int C = a.c1 + a.c2;
    switch (ck) {
        case CK_PERS: return halo && a.N <= 32 && (C == HC || C == 2 * HC);
        case CK_HALO32: return halo;
        case CK_HALO64: return halo;
        case CK_GEMM64:
        case CK_GEMM128: return true;
        case CK_GEMM64W: return a.N >= 128;
        case CK_GEMM128W: return a.N >= 64;
        case CK_PERS16: return halo && a.N <= 16 && C == HC;   // narrow outputs (the 2-channel head)
        case CK_DL64: return halo && a.N > 32 && a.gmode == G_CONV;   // forward only
        case CK_UPP: return upconv_ok(a);
        case CK_GPF64: return gemm_pf_ok(a);
        case CK_GPF128: return gemm_pf_ok(a) && a.N >= 128;
        case CK_SMALLC: return smallc_ok(a);
        case CK_FIRST2: return first2_ok(a);
    }
    return false;
}

static int ck_default(const GemmArgs& a) {
    if (halo_ok(a)) {
        if (ck_applicable(a, CK_PERS)) return CK_PERS;
        return a.N <= 32 ? CK_HALO32 : CK_HALO64;
    }
    if (first2_ok(a)) return CK_FIRST2;
    if (smallc_ok(a)) return CK_SMALLC;
    return a.N <= 32 ? CK_GEMM128 : CK_GEMM64;
}

template <int FLIP, int EPI>
static void launch_halo_ck(const GemmArgs& a, hipStream_t s, unsigned long long* wc, int ck) {
    const int C = a.c1 + a.c2;
    if (ck == CK_PERS) {
        if (C == HC)
            launch_pers<32, FLIP, EPI, 1>(a, s, wc);
        else
            launch_pers<32, FLIP, EPI, 2>(a, s, wc);
    } else if (ck == CK_PERS16) {
        launch_pers<16, FLIP, EPI, 1>(a, s, wc);
    } else if (ck == CK_HALO32) {
        launch_single<32, FLIP, EPI>(a, s, wc);
    } else if (ck == CK_DL64) {
        if constexpr (FLIP == 0 && EPI == E_FWD) {
            const int ntiles = ((a.Ho + DTY - 1) / DTY) * ((a.Wo + DTX - 1) / DTX) * a.B;
            TIMED_LAUNCH("k_conv", s, k_conv3_dl, dim3(ntiles, (a.N + 63) / 64), dim3(512), 0, s, a, wc);
        } else {
            launch_single<64, FLIP, EPI>(a, s, wc);   // not applicable (ck_applicable excludes it)
        }
    } else {
        launch_single<64, FLIP, EPI>(a, s, wc);
    }
}

static int launch_ck(const GemmArgs& a, hipStream_t s, int ck, unsigned long long* wc) {
    switch (ck) {
        case CK_PERS:
        case CK_PERS16:
        case CK_HALO32:
        case CK_HALO64:
        case CK_DL64:
            if (a.gmode == G_CONVT)
                launch_halo_ck<1, E_ACC>(a, s, wc, ck);
            else
                launch_halo_ck<0, E_FWD>(a, s, wc, ck);
            break;
        case CK_GPF64:
        case CK_GPF128: {
            const dim3 grid((unsigned)((a.M + 63) / 64), (a.N + (ck == CK_GPF64 ? 63 : 127)) / (ck == CK_GPF64 ? 64 : 128));
            if (ck == CK_GPF64)
                TIMED_LAUNCH("k_conv", s, (k_gemm_pf<64, 64, 2, 2>), grid, dim3(256), 0, s, a, wc);
            else
                TIMED_LAUNCH("k_conv", s, (k_gemm_pf<64, 128, 2, 2>), grid, dim3(256), 0, s, a, wc);
            break;
        }
        case CK_UPP:
            switch (a.c1) {
                case 64: launch_upconv_k<64>(a, s, wc); break;
                case 128: launch_upconv_k<128>(a, s, wc); break;
                default: launch_upconv_k<256>(a, s, wc); break;
            }
            break;
        case CK_FIRST2: {
            const long nseg = (long)a.B * a.Ho * ((a.Wo + 15) / 16);
            const dim3 grid((unsigned)std::max<long>(1, std::min<long>(4096, (nseg + 3) / 4)));
            switch (a.N / 16) {
                case 1: TIMED_LAUNCH("k_conv", s, k_conv3_first2<1>, grid, dim3(256), 0, s, a, wc); break;
                case 2: TIMED_LAUNCH("k_conv", s, k_conv3_first2<2>, grid, dim3(256), 0, s, a, wc); break;
                case 3: TIMED_LAUNCH("k_conv", s, k_conv3_first2<3>, grid, dim3(256), 0, s, a, wc); break;
                default: TIMED_LAUNCH("k_conv", s, k_conv3_first2<4>, grid, dim3(256), 0, s, a, wc); break;
            }
            break;
        }
        case CK_SMALLC: {
            const dim3 grid((unsigned)std::min<long>(2048, (a.M * (a.N / 8) + 255) / 256));
            switch (a.c1) {
                case 1: TIMED_LAUNCH("k_conv", s, k_conv3_smallc<1>, grid, dim3(256), 0, s, a, wc); break;
                case 2: TIMED_LAUNCH("k_conv", s, k_conv3_smallc<2>, grid, dim3(256), 0, s, a, wc); break;
                case 3: TIMED_LAUNCH("k_conv", s, k_conv3_smallc<3>, grid, dim3(256), 0, s, a, wc); break;
                default: TIMED_LAUNCH("k_conv", s, k_conv3_smallc<4>, grid, dim3(256), 0, s, a, wc); break;
            }
            break;
        }
        default: {
            const int shape = ck == CK_GEMM128 ? 1 : ck == CK_GEMM64W ? 2 : ck == CK_GEMM128W ? 3 : 0;
            switch (a.gmode) {
                case G_CONV: launch_gemm_pick<G_CONV>(a, s, wc, shape); break;
                case G_CONVT: launch_gemm_pick<G_CONVT>(a, s, wc, shape); break;
                case G_UP: launch_gemm_pick<G_UP>(a, s, wc, shape); break;
                case G_UPT: launch_gemm_pick<G_UPT>(a, s, wc, shape); break;
                default: return fail(HELM_EINVAL, "gemm: gather mode %d", a.gmode);
            }
        }
    }
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

namespace {
struct TuneKey {
    int v[16];
    bool operator<(const TuneKey& o) const {
        for (int i = 0; i < 16; ++i)
            if (v[i] != o.v[i]) return v[i] < o.v[i];
        return false;
    }
};
std::map<TuneKey, int> g_tuned;
std::mutex g_tune_mutex;
bool g_tune_on = true;
int g_force = -1;   // pinned kernel (where applicable), -1 for none

TuneKey tune_key(const GemmArgs& a) {
    TuneKey k{};
    int i = 0;
    k.v[i++] = a.gmode;
    k.v[i++] = a.epi;
    k.v[i++] = a.stride;
    k.v[i++] = a.c1;
    k.v[i++] = a.c2;
    k.v[i++] = a.abs2 == 0;
    k.v[i++] = a.N;
    k.v[i++] = a.K;
    k.v[i++] = a.B;
    k.v[i++] = a.Hi;
    k.v[i++] = a.Wi;
    k.v[i++] = a.Ho;
    k.v[i++] = a.Wo;
    k.v[i++] = (a.resid != nullptr) | (a.outf != nullptr) << 1 | (a.bmap != nullptr) << 2 | (a.relu != 0) << 3;
    k.v[i++] = a.st != nullptr;
    return k;
}

bool capturing_stream(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Times every applicable candidate (1 warm-up + 3 timed launches each).
int tune(const GemmArgs& a, hipStream_t s, int* best) {
    hipEvent_t e0, e1;
    HELM_HIP(hipEventCreate(&e0));
    HELM_HIP(hipEventCreate(&e1));
    float best_ms = 0;
    *best = ck_default(a);
    for (int ck = 0; ck < CK_COUNT; ++ck) {
        if (!ck_applicable(a, ck)) continue;
        int rc = launch_ck(a, s, ck, nullptr);
        if (rc) return rc;
        HELM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r)
            if ((rc = launch_ck(a, s, ck, nullptr))) return rc;
        HELM_HIP(hipEventRecord(e1, s));
        HELM_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HELM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ck == ck_default(a)) ms *= 0.9f;     // a candidate must beat the rule by 10% (stable choices)
        if (best_ms == 0 || ms < best_ms) {
            best_ms = ms;
            *best = ck;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return HELM_OK;
}
}  // namespace

int launch_gemm(const GemmArgs& a, hipStream_t s) {
    if (a.K % KC != 0) return fail(HELM_EINVAL, "gemm: K=%d not a multiple of %d", a.K, KC);
    if (a.M * (long)std::max(1, a.N) >= (1L << 31) || (long)a.B * a.Hi * a.Wi >= (1L << 31))
        return fail(HELM_EINVAL, "gemm: grid of %ld rows too large for 32-bit pixel indexing", a.M);
    if (a.M <= 0 || a.N <= 0) return HELM_OK;
    int ck = ck_default(a);
    const bool tunable = (a.epi == E_FWD || a.epi == E_UPFWD) && a.out != nullptr;
    int forced = -1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        forced = g_force;
    }
    if (forced >= 0 && ck_applicable(a, forced)) {
        ck = forced;
    } else if (tunable) {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        if (g_tune_on) {
            const TuneKey key = tune_key(a);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                ck = it->second;
            } else if (!capturing_stream(s)) {
                int rc = tune(a, s, &ck);
                if (rc) return rc;
                g_tuned[key] = ck;
            }
        }
    }
    return launch_ck(a, s, ck, WORK_COUNTER("k_conv", s));
}

// Tuned choices to / from a text file (one shape per line: 16 key fields, then
// the kernel), so that another process can launch exactly the same kernels.
int conv_autotune_file(const char* path, int save) {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    if (save) {
        FILE* f = fopen(path, "w");
        if (!f) return fail(HELM_EINVAL, "helm_autotune_file: cannot write %s", path);
        for (const auto& kv : g_tuned) {
            for (int i = 0; i < 16; ++i) fprintf(f, "%d ", kv.first.v[i]);
            fprintf(f, "%d\n", kv.second);
        }
        fclose(f);
        return HELM_OK;
    }
    FILE* f = fopen(path, "r");
    if (!f) return fail(HELM_EINVAL, "helm_autotune_file: cannot read %s", path);
    for (;;) {
        TuneKey k{};
        int ck = 0, got = 0;
        for (int i = 0; i < 16; ++i) got += fscanf(f, "%d", &k.v[i]);
        got += fscanf(f, "%d", &ck);
        if (got != 17) break;
        if (ck < 0 || ck >= CK_COUNT) {
            fclose(f);
            return fail(HELM_EINVAL, "helm_autotune_file: bad kernel id %d in %s", ck, path);
        }
        g_tuned[k] = ck;
    }
    fclose(f);
    return HELM_OK;
}

int conv_force(int kernel, int* count) {
    if (count) *count = CK_COUNT;
    if (kernel < -1 || kernel >= CK_COUNT)
        return fail(HELM_EINVAL, "helm_conv_force: kernel %d outside -1 .. %d", kernel, CK_COUNT - 1);
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_force = kernel;
    return HELM_OK;
}

int conv_autotune(int enable, int* tuned) {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    if (enable == 0 || enable == 1) g_tune_on = enable == 1;
    if (enable == 2) g_tuned.clear();
    if (tuned) *tuned = (int)g_tuned.size();
    return HELM_OK;
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

// ------------------------------------------------------------------ weight gradient, stride-1 3x3 layers
// dW[n][tap][c] = sum over pixels p of g[p][n] x[p + shift(tap)][c].  A block owns
// 32 output channels (n0..), one 32-channel chunk of the input (c0..) and the
// 16 x 16 pixel tiles t = blockIdx.x, blockIdx.x + gridDim.x, ...  Per tile it
// stages g transposed ([n][pixel]) and the 18 x 18 input patch transposed in
// three column-shifted copies ([kx][c][row][col]), so that every MFMA operand
// fragment (eight consecutive pixels of one channel) is one aligned 16-byte LDS
// read; the reduction over pixels is the MFMA's K.  Wave w accumulates the
// 16 x 16 block (n-tile w/2, c-tile w%2) of all nine taps; the block writes its
// sum to part[blockIdx.x] and a fixed-order fold adds the partials.
constexpr int WG3_GLD = HT * HT + 8;      // gT row: 256 pixels (+ pad)
constexpr int WG3_XLD = HP * HT + 8;      // xT row: 18 patch rows x 16 columns (+ pad)

__global__ __launch_bounds__(256) void k_wgrad3(WgradArgs a) {
    __shared__ bf16 gT[32][WG3_GLD];
    __shared__ bf16 xT[3][32][WG3_XLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n0 = blockIdx.y * 32, c0 = blockIdx.z * 32;
    const int tiles_x = (a.Wg + HT - 1) / HT, tiles_y = (a.Hg + HT - 1) / HT, tps = tiles_x * tiles_y;
    const int ntiles = a.B * tps;
    const int C = a.c1 + a.c2;
    const bool s2 = c0 >= a.c1;
    const bf16* xs = s2 ? a.a2 : a.a1;
    const int cs = s2 ? a.c2 : a.c1, cc = s2 ? c0 - a.c1 : c0;
    const long xbs = s2 ? a.abs2 : a.abs1;
    const int nt = wave >> 1, ct = wave & 1;
    f32x4 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = t / tps, ty0 = ((t / tiles_x) % tiles_y) * HT, tx0 = (t % tiles_x) * HT;
        // g tile (256 pixels x 32 channels) -> gT
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sg = tid + q * 256, pix = sg >> 2, sub = sg & 3;
            const int y = ty0 + (pix >> 4), x = tx0 + (pix & 15), n = n0 + sub * 8;
            bf16x8 v = zero8();
            if (y < a.Hg && x < a.Wg && n < a.M) {
                const bf16* src = a.g + (((long)b * a.Hg + y) * a.Wg + x) * a.Cg + n;
                if (n + 8 <= a.M) {
                    v = ld8(src);
                } else {
                    for (int e = 0; e < 8 && n + e < a.M; ++e) v[e] = src[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) gT[sub * 8 + e][pix] = v[e];
        }
        // input patch (18 x 18 pixels x 32 channels) -> three column-shifted transposed copies
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int sg = tid + q * 256;
            if (sg >= HP * HP * 4) break;
            const int pix = sg >> 2, sub = sg & 3;
            const int py = pix / HP, px = pix - py * HP;
            const int yi = ty0 + py - 1, xi = tx0 + px - 1;
            const bf16x8 v = (yi >= 0 && yi < a.Hi && xi >= 0 && xi < a.Wi)
                                 ? ld8(xs + b * xbs + ((long)yi * a.Wi + xi) * cs + cc + sub * 8)
                                 : zero8();
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int col = px - kx;
                if (col < 0 || col >= HT) continue;
#pragma unroll
                for (int e = 0; e < 8; ++e) xT[kx][sub * 8 + e][py * HT + col] = v[e];
            }
        }
        __syncthreads();
        // eight K-steps of 32 pixels (two tile rows)
        const int gq = lane >> 4;
#pragma unroll 2
        for (int ks = 0; ks < 8; ++ks) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&gT[nt * 16 + (lane & 15)][ks * 32 + gq * 8]);
            const int r = 2 * ks + (gq >> 1), col0 = 8 * (gq & 1);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ky = tap / 3, kx = tap % 3;
                const bf16x8 fb =
                    *reinterpret_cast<const bf16x8*>(&xT[kx][ct * 16 + (lane & 15)][(r + ky) * HT + col0]);
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[tap], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // acc[tap][e] = dW[n = n0 + 16 nt + 4 (l/16) + e][tap][c = c0 + 16 ct + l%16]
    float* part = a.part + (long)blockIdx.x * a.M * a.Npad;
    const int c = c0 + ct * 16 + (lane & 15);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int n = n0 + nt * 16 + (lane >> 4) * 4 + e;
            if (n < a.M) part[(long)n * a.Npad + tap * C + c] = acc[tap][e];
        }
}

static bool wgrad3_ok(const WgradArgs& a) {
    return a.mode == G_CONV && a.stride == 1 && a.c1 % 32 == 0 && a.c2 % 32 == 0 && a.c1 > 0 &&
           a.Hg == a.Hi && a.Wg == a.Wi && a.Npad >= 9 * (a.c1 + a.c2);
}

// Weight gradient into max_split partial slabs of [M][Npad] floats; *nsplit is
// set to the number of slabs written (the fold sums exactly those).
int launch_wgrad(WgradArgs a, int max_split, hipStream_t s, int* nsplit) {
    if (max_split < 1) return fail(HELM_EINVAL, "wgrad: no partial-sum space");
    if (wgrad3_ok(a)) {
        const int tiles = ((a.Hg + HT - 1) / HT) * ((a.Wg + HT - 1) / HT) * a.B;
        const int nb = (a.M + 31) / 32, cb = (a.c1 + a.c2) / 32;
        const int gx = std::max(1, std::min({tiles, max_split, std::max(1, 512 / (nb * cb))}));
        TIMED_LAUNCH("k_wgrad", s, k_wgrad3, dim3(gx, nb, cb), dim3(256), 0, s, a);
        HELM_CHECK_LAUNCH();
        *nsplit = gx;
        return HELM_OK;
    }
    // general path: about 2048 workgroups in flight, pixel range split into chunks
    const long tiles = (long)((a.Npad + WG_BN - 1) / WG_BN) * ((a.M + WG_BM - 1) / WG_BM);
    int ns = (int)std::max<long>(1, std::min<long>(std::min<long>(64, max_split), 2048 / std::max<long>(1, tiles)));
    a.pchunk = (int)((a.P + ns - 1) / ns);
    a.pchunk = (a.pchunk + 31) / 32 * 32;
    ns = (int)((a.P + a.pchunk - 1) / a.pchunk);
    dim3 grid((a.Npad + WG_BN - 1) / WG_BN, (a.M + WG_BM - 1) / WG_BM, ns);
    TIMED_LAUNCH("k_wgrad", s, k_wgrad, grid, dim3(256), 0, s, a);
    HELM_CHECK_LAUNCH();
    *nsplit = ns;
    return HELM_OK;
}

}  // namespace helm
