// BF16 MFMA convolution kernels of the encoder-solver networks (gfx950).
#pragma once
#include "internal.h"

namespace helm {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Row space of every GEMM is a pixel grid (b, y, x) of B x Ho x Wo; how the
// A operand (pixels x K) is gathered:
enum GatherMode {
    G_CONV = 0,   // 3x3 conv, pad 1, stride s: k = tap*C + c, input (s*y+ky-1, s*x+kx-1)
    G_CONVT = 1,  // transposed 3x3 (data gradient): k = tap*C + c, source (y+1-ky)/s when divisible
    G_UP = 2,     // 1x1 on the up-conv input: k = c at (y, x)
    G_UPT = 3,    // up-conv data gradient: k = (2a+d)*C + c at (2y+a, 2x+d)
};
// What happens to D[m][n] (+ bias etc.):
enum EpiMode {
    E_FWD = 0,    // out[m][n] = act(D + bias[n] (+ resid[m][n])), bf16 (+ optional fp32 copy); out may be null
    E_UPFWD = 1,  // n = (2a+d)*Cout + co -> out[(b, 2y+a, 2x+d)][co] = relu(D + bias[co])
    E_ACC = 2,    // fp32 accumulate: n < n1 -> acc1[m][n], else acc2[m][n-n1]
};


struct GemmArgs {
    int gmode;       // GatherMode
    const bf16* a1;
    const bf16* a2;
    int c1, c2;      // channels of the two concatenated sources (c2 = 0: one source)
    long abs1, abs2; // batch strides (elements) of the sources (0: broadcast)
    int B, Hi, Wi;   // spatial size of the gathered tensors
    int Ho, Wo;      // row grid
    int stride;
    int K;           // GEMM depth (multiple of 32; padded with zeros past 9*C for small C)
    int kvalid;      // number of real k's
    const bf16* w;   // [N][K] bf16
    int N;
    int epi;
    const float* bias;
    const bf16* resid;
    int relu;
    bf16* out;
    float* outf;
    float* acc1;
    float* acc2;
    int n1;
    long M;
    const RhsState* st;  // optional: skip row tiles of samples whose RHS is inactive
    int rhs0;
    const bf16* bmap;    // E_FWD: [Ho][Wo][N] added instead of bias (same for every sample)
};

struct WgradArgs {
    const bf16* g;   // masked output gradient, [B][Hg][Wg][Cg]
    int Hg, Wg, Cg;
    const bf16* a1;  // forward input sources (as in GemmArgs)
    const bf16* a2;
    int c1, c2;
    long abs1, abs2;
    int B, Hi, Wi;
    int stride;
    int mode;        // G_CONV (conv weights [Cout][9][C]) or G_UP (weights [2][2][Cout][C])
    int M;           // rows of the weight gradient: Cout (conv) or 4*Cout (up)
    int N;           // columns: 9*C (conv) or C (up)
    int Npad;        // N rounded up to the tile
    long P;          // reduction length (pixels)
    int pchunk;      // pixels per split (set by launch_wgrad)
    float* part;     // [nsplit][M][Npad]
};

int launch_gemm(const GemmArgs& a, hipStream_t s);

// Fused residual block y = x + conv2(ReLU(conv1(x) + b1)) + b2, 32 channels,
// stride 1 (inference); weights in the forward layout [32][K] (k = tap*32 + c).
struct ResArgs {
    const bf16* x;       // [B][H][W][32], also the residual
    int B, H, W;
    const bf16* w1;
    int K1;
    const float* b1;
    const bf16* w2;
    int K2;
    const float* b2;
    bf16* out;           // [B][H][W][32]
    const RhsState* st;  // optional: skip samples whose RHS is inactive
    int rhs0;
};
int launch_resblock32(const ResArgs& a, hipStream_t s);

// Fused first layer and level-0 context convolution of the solver (inference):
// out = ReLU(conv_h(h0) + bmap) with h0 = ReLU(conv0(r) + b0) computed per tile
// in LDS, so h0 never goes to memory.  r has 2 channels, h0 and out 32.
struct FirstCtxArgs {
    const bf16* r;       // [B][H][W][2]
    int B, H, W;
    const bf16* w0;      // first layer [32][K0], k = tap * 2 + c (K0 >= 32, zero past 18)
    int K0;
    const float* b0;     // [32]
    const bf16* wh;      // the context convolution's h part [32][Kh], k = tap * 32 + c
    int Kh;
    const bf16* bmap;    // [H][W][32]: its z part plus bias, per pixel
    bf16* out;           // [B][H][W][32]
    const RhsState* st;  // optional: skip samples whose RHS is inactive
    int rhs0;
};
int launch_first_ctx(const FirstCtxArgs& a, hipStream_t s);
// enable: 1 on, 0 off (built-in rule), 2 forget the tuned shapes; -1 query only.
int conv_autotune(int enable, int* tuned);
int conv_autotune_file(const char* path, int save);
int conv_force(int kernel, int* count);
// Weight gradient into at most max_split partial slabs [M][Npad] at a.part;
// *nsplit receives the number written (a.pchunk is chosen here).
int launch_wgrad(WgradArgs a, int max_split, hipStream_t s, int* nsplit);

}  // namespace helm
