/*
 * helm.h -- C ABI of libhelm, a gfx950 library for repeated 2D Helmholtz
 * solves preconditioned by a shifted-Laplacian multigrid cycle and by an
 * encoder-solver convolutional network (Goren & Treister, "Physics-guided Full
 * Waveform Inversion using Encoder-Solver Convolutional Neural Networks").
 *
 * Conventions (every entry point):
 *   - grids are row-major [nz][nx], x (columns) fastest, row 0 at the surface;
 *     nx must be even (two nodes are loaded per lane);
 *   - complex arrays are interleaved (re, im); "c64" = 2 x float,
 *     "c128" = 2 x double; a batch of right-hand sides is stored back to back
 *     (batch outermost);
 *   - every data pointer is a DEVICE pointer owned by the caller unless the
 *     comment says "host"; the library never frees caller memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream); work
 *     is enqueued on it, and entry points return once their host-visible
 *     outputs are written (helm_solve reads one small per-RHS status block back
 *     to the host per restart cycle);
 *   - return codes: HELM_OK, HELM_NOT_CONVERGED (soft: per-RHS status filled),
 *     or a negative hard error; helm_last_error() gives the message;
 *   - handles are not thread-safe; distinct handles may be used from distinct
 *     threads.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK 0
#define HELM_NOT_CONVERGED 1
#define HELM_EINVAL (-1)
#define HELM_ENOMEM (-2)
#define HELM_EHIP (-3)
#define HELM_ENAN (-4)

#define HELM_C64 0
#define HELM_C128 1

#define HELM_PRECOND_MG 0     /* M = V_SL, the shifted-Laplacian V-cycle        */
#define HELM_PRECOND_NONE 1   /* M = I                                          */
#define HELM_PRECOND_CNN 2    /* M = SolverNet only                             */
#define HELM_PRECOND_CNN_VU 3 /* M_VU(r) = e0 + V_SL(r - H e0), e0 = SolverNet(r) */

typedef struct helm_op* helm_op_t;
typedef struct cnn_net* cnn_net_t;

/* Options of helm_setup.  Zero-initialised fields take the defaults. */
typedef struct {
    double hz;            /* vertical spacing; <= 0 means hz = h                 */
    double sl_beta;       /* shift beta of eq. (3.12); <= 0 means 0.5            */
    int sl_no_gamma;      /* 1: literal P = -Lap - w^2 m (1 - beta i) (no gamma) */
    int mg_levels;        /* <= 0 means 3 (Sec. 3.4); 1..4 accepted              */
    int coarse_degree;    /* degree of the coarsest-level polynomial; <= 0: 20   */
    double jacobi_weight; /* damped-Jacobi weight; <= 0 means 0.8                */
} helm_setup_opts;

/*
 * helm_setup -- operator H(m, omega) of eq. (3.1)-(3.2) and its shifted-
 * Laplacian hierarchy (eq. (3.12)).
 *   kappa2 [nz][nx] float: squared slowness m = 1/c^2 (device);
 *   gamma  [nz][nx] float: attenuation fraction (absorbing layer) (device);
 *   omega: angular frequency; h: horizontal spacing (opt->hz vertical).
 * H u = (2u - u_W - u_E)/hx^2 + (2u - u_N - u_S)/hz^2 - omega^2 m (1 - i gamma) u,
 * with zero values outside the grid.  The handle copies kappa2 and gamma; the
 * caller may free them afterwards.  Errors: HELM_EINVAL (nz, nx < 4, odd nx,
 * non-positive h or omega), HELM_ENOMEM, HELM_EHIP.
 */
int helm_setup(const float* kappa2, const float* gamma, int nz, int nx, double omega, double h,
               const helm_setup_opts* opt, void* stream, helm_op_t* out);
void helm_destroy(helm_op_t op);
/* Grid size of an operator (host outputs; any may be NULL). */
int helm_op_info(helm_op_t op, int* nz, int* nx, double* omega, double* hx, double* hz);

/*
 * helm_matvec -- v = H u (adjoint = 0) or v = H^* u (adjoint = 1) for nrhs
 * vectors [nrhs][nz][nx] of type dtype (HELM_C64 or HELM_C128).  u and v must
 * not overlap.  Eq. (3.2); H^* = conj(H) because H is complex symmetric (Sec. 4.3).
 * nrhs = 0 is a no-op (u and v may then be NULL).
 */
int helm_matvec(helm_op_t op, const void* u, void* v, int nrhs, int dtype, int adjoint, void* stream);

/* Options of helm_solve.  Zero-initialised fields take the defaults. */
typedef struct {
    int precond;          /* HELM_PRECOND_*; default HELM_PRECOND_MG             */
    int restart;          /* Krylov cycle length m; <= 0: 20 (MG/NONE), 10 (CNN) */
    int maxit;            /* iteration cap per RHS; <= 0: 300 (Sec. 5.7)         */
    int adjoint;          /* 1: solve H^* x = b by conjugation (eq. (4.4)-(4.8)) */
    int krylov_dtype;     /* HELM_C64 (default) or HELM_C128 basis vectors       */
    int x0_given;         /* 1: x holds the initial guess; 0: start from x = 0   */
    int use_graph;        /* 1: replay each restart cycle from a captured graph  */
    int reorth;           /* 1: second Gram-Schmidt pass when ||w|| drops by 0.7 */
    cnn_net_t net;        /* network for the CNN preconditioners                 */
    int streams;          /* 2: the CNN preconditioners apply each operator's    */
                          /* batch as two halves on two streams (the caller's    */
                          /* and a library stream, joined by events, also under  */
                          /* graph capture), so that the halves' kernels overlap;*/
                          /* with the same convolution kernels, the same results;*/
                          /* 0 or 1: one stream                                  */
} helm_solve_opts;

/*
 * helm_solve -- flexible GMRES(m), right preconditioned, for a batch of
 * systems H_{op(r)} x_r = b_r (Sec. 3.4, eq. (3.14)).
 *   ops[nops]: operators; rhs_op[nrhs] (host): operator index of each RHS,
 *     non-decreasing (RHS grouped by operator); NULL puts every RHS on ops[0];
 *   rhs: c64 right-hand sides, back to back in RHS order (device);
 *   x:   c128 solutions, same layout (device; in: initial guess if x0_given);
 *   iters, relres, status [nrhs] (host outputs, may be NULL): iterations,
 *     FP64 ||b - H x|| / ||b||, and per-RHS HELM_OK / HELM_NOT_CONVERGED /
 *     HELM_ENAN.
 * Stopping: relres <= tol with the residual recomputed in FP64 from the c128
 * iterate at every restart; b = 0 gives x = 0.  nrhs = 0 is a no-op that
 * returns HELM_OK (rhs and x may then be NULL).  Returns HELM_OK when every RHS
 * converged, HELM_NOT_CONVERGED otherwise, or a hard error.
 */
int helm_solve(const helm_op_t* ops, int nops, const int* rhs_op, const void* rhs, void* x, int nrhs,
               double tol, const helm_solve_opts* opt, int* iters, double* relres, int* status,
               void* stream);

/*
 * helm_vcycle -- e = V_SL(f): one shifted-Laplacian V-cycle from e = 0
 * (Sec. 3.4, three levels) for nrhs c64 vectors (device).  Linear in f.
 * nrhs = 0 is a no-op (f and e may then be NULL).
 */
int helm_vcycle(helm_op_t op, const void* f, void* e, int nrhs, void* stream);
/*
 * helm_resample -- bilinear resampling of a nodal field in [nz][nx] onto
 * out [mz][mx] covering the same extent (output node (I, K) sits at input
 * coordinates I (nz-1)/(mz-1), K (nx-1)/(mx-1); FP64 weights, float I/O, both
 * device).  The inversion driver uses it to put the model and the absorbing
 * layer on the grid with 10 points per wavelength at a window's highest
 * frequency, where the network is retrained (Sec. 5, retraining details).
 * in and out must not overlap.
 */
int helm_resample(const float* in, int nz, int nx, float* out, int mz, int mx, void* stream);
/*
 * helm_vcycle_noalloc -- helm_vcycle for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and result, with the cycle's scratch
 * (coarse-level right-hand sides and corrections, coarsest-level FP64
 * buffers: 2 x 8 B x nrhs x (N_1 + N_2) + 3 x 16 B x nrhs x N_2 for three
 * levels, N_l = nodes of level l, each piece rounded up to 256 B) in a fixed
 * device array of helm_vcycle_noalloc_max_bytes() = 32 MiB per GPU that the
 * library holds until the process ends.  The call allocates nothing; it
 * returns HELM_EINVAL when the scratch would exceed the array (512 KiB per
 * right-hand side of a 256 x 256 grid: at most 64 of them per call).  Every call on a GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (other streams or threads) race and must not be issued.
 */
int helm_vcycle_noalloc(helm_op_t op, const void* f, void* e, int nrhs, void* stream);
size_t helm_vcycle_noalloc_max_bytes(void);
/* Roots of the coarsest-level polynomial, in application order (host, c128 [*n]). */
int helm_coarse_roots(helm_op_t op, double* roots, int* n);

/* ------------------------------------------------------------------------
 * Encoder-solver network (Sec. 3.4, 4.1-4.3, Fig. 1).  Architecture: four
 * levels of widths w[0..3] (default 32, 64, 128, 256); the encoder maps
 * [omega^2 hx hz m, gamma] to context maps z_0..z_3 (once per operator and
 * weight version), the solver maps the scaled residual [Re, Im](s r),
 * s = sqrt(N)/||r||, with z_l concatenated at every level, to hx hz s e.
 * BF16 activations (NHWC) and weights, FP32 accumulation and master weights.
 * Grids must have nz, nx divisible by 8.
 * ------------------------------------------------------------------------ */
typedef struct {
    int widths[4];   /* <= 0: default; multiples of 32 */
    int down_res;    /* residual blocks per encoder level on the way down; <= 0: 2 */
} cnn_arch;

/* cnn_create -- network with He-normal weights drawn from Philox-4x32-10 (key = seed). */
int cnn_create(const cnn_arch* arch, uint64_t seed, cnn_net_t* out);
void cnn_destroy(cnn_net_t net);
/* Weights, Adam moments and step count to / from a file (host path). */
int cnn_save(cnn_net_t net, const char* path);
int cnn_load(const char* path, cnn_net_t* out);
/* Flat FP32 parameters, layer by layer, W then b (host buffers of cnn_num_params floats). */
int cnn_num_params(cnn_net_t net, long* count);
int cnn_get_params(cnn_net_t net, float* host);
int cnn_set_params(cnn_net_t net, const float* host);
int cnn_get_grad(cnn_net_t net, float* host);
int cnn_zero_grad(cnn_net_t net);

/* Raw network: out = SolverNet(rin; EncoderNet(op)), rin and out FP32
 * [B][nz][nx][2] (device). */
int cnn_forward(cnn_net_t net, helm_op_t op, const float* rin, float* out, int B, void* stream);
/* e = M_net(r) = hx hz net(s r) / s for nrhs c64 vectors (device); Sec. 3.4.
 * nrhs = 0 is a no-op (r and e may then be NULL). */
int cnn_precond_apply(cnn_net_t net, helm_op_t op, const void* r, void* e, int nrhs, void* stream);
/* MSE loss of eq. (4.2) on B pairs (r, e) (c64, device) and its gradient,
 * accumulated into the network's gradient buffer; loss to host (may be NULL). */
int cnn_loss_grad(cnn_net_t net, helm_op_t op, const void* r, const void* e, int B, double* loss, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the accumulated gradient, which it zeroes. */
int cnn_adam_step(cnn_net_t net, double lr, void* stream);
/* Training pairs of eq. (4.3) for samples first .. first+npairs-1: x ~ CN(0,1)
 * (Philox stream = sample index, key (seed, 0xDA7A)), b = H x, x~ = GMRES with
 * the V-cycle for k ~ U{1..10} iterations, e = x - x~, r = H e (c64, device). */
int cnn_make_pairs(helm_op_t op, int first, int npairs, uint64_t seed, void* r, void* e, void* stream);
/* One data epoch of Alg. 2 on r, e [2*npairs][N] (device): appends the pairs
 * spawned by the first npairs at index npairs .. 2*npairs-1. */
int cnn_alg2_epoch(cnn_net_t net, helm_op_t op, void* r, void* e, int npairs, void* stream);

/*
 * Single-layer hooks (test and tuning): one 3x3 convolution (kind 0: stride 1
 * or 2, sources x1 [B][H][W][c1] and optionally x2 [B or 1][H][W][c2]
 * concatenated after x1, weights [cout][3][3][c1+c2]) or one 2x2 up-convolution
 * (kind 1: weights [2][2][cout][c1]) through the same BF16 MFMA kernels the
 * networks use.  All arrays are FP32 HOST buffers; inputs are rounded to BF16.
 * Forward: out = act(conv + b (+ resid)).  Backward: given the forward output y
 * (for the ReLU mask) and dL/dy, the gradients w.r.t. x1, x2 (per sample), W, b.
 */
int cnn_layer_forward(int kind, int stride, int B, int H, int W, int c1, int c2, int bcast2, int cout,
                      const float* x1, const float* x2, const float* w, const float* b, const float* resid, int relu,
                      float* out);
int cnn_layer_backward(int kind, int stride, int B, int H, int W, int c1, int c2, int bcast2, int cout,
                       const float* x1, const float* x2, const float* w, const float* y, int relu, const float* gout,
                       float* gx1, float* gx2, float* gw, float* gb);
/* Fused 32-channel residual block out = x + conv2(ReLU(conv1(x) + b1)) + b2
 * (stride 1, zero padding; weights [32][3][3][32], FP32 HOST buffers, x and
 * out [B][H][W][32], inputs rounded to BF16, out rounded to BF16), the kernel
 * that inference uses for the networks' first-level residual blocks. */
int cnn_layer_resblock(int B, int H, int W, const float* x, const float* w1, const float* b1, const float* w2,
                       const float* b2, float* out);

typedef struct {
    int npairs;            /* plain training: pairs generated by eq. (4.3); <= 0: 2000 */
    int batch;             /* <= 0: 16 */
    int steps;             /* optimiser steps; <= 0: 200 */
    double lr;             /* Adam learning rate; <= 0: 1e-4 */
    int alg2_initial;      /* > 0: Alg. 2 with this initial dataset size */
    int alg2_data_epochs;  /* Alg. 2: epochs that also generate data */
    int alg2_epochs;       /* Alg. 2: total epochs */
    int* steps_done;       /* host output, may be NULL */
    int* dataset_size;     /* host output, may be NULL */
} cnn_train_opts;

/* cnn_precond_train -- generate pairs on op's medium and train (Sec. 4.1) or
 * retrain with Alg. 2 (Sec. 4.2); loss per step to loss_hist (host, steps). */
int cnn_precond_train(cnn_net_t net, helm_op_t op, const cnn_train_opts* opt, uint64_t seed, float* loss_hist,
                      void* stream);

/* ------------------------------------------------------------------------
 * Full-waveform-inversion misfit and gradient (eq. (3.5), (3.10), (4.4)-(4.8)).
 * ------------------------------------------------------------------------ */
/*
 * fwi_misfit_grad -- Phi = 1/2 sum_{f,s} || R u_fs - d_fs ||^2 with
 * u_fs = H_f^{-1} g_s, and dPhi/dm for the squared slowness m of the media.
 *   ops[nfreq]: one operator per frequency, all on the same grid and built
 *     from the same m and gamma (checked on the device: HELM_EINVAL
 *     otherwise; the gradient is taken with respect to that m, each
 *     operator's own omega entering it);
 *   src_idx[nsrc], rec_idx[nrec] (host): flat node indices row * nx + col; the
 *     source of s is the grid delta g_s = e_src / (hx hz); receivers sample the
 *     wavefield at their nodes and must be distinct;
 *   dobs: observed data, c64 [nfreq][nsrc][nrec] (device);
 *   tol, opt: the solver tolerance and options of both solve batches
 *     (opt->adjoint must be 0; opt->x0_given is ignored);
 *   misfit (host): Phi, accumulated in FP64;
 *   grad: dPhi/dm = sum_f w_f^2 sum_s Re(conj(lambda_fs) (1 - i gamma) u_fs),
 *     lambda_fs = H_f^{-*} R^T (R u_fs - d_fs) by conjugation (eq. (4.8)),
 *     FP64 accumulation, written as float [nz][nx] (device);
 *   iters (host, may be NULL): [2][nfreq][nsrc] iterations of the forward
 *     then the adjoint solves.
 * All nfreq * nsrc forward solves go into one helm_solve batch, then all
 * adjoint solves.  Workspace (two c128 and one c64 field per (f, s)) comes
 * from a device pool that the FWI entry points share and keep between calls
 * (fwi_release_workspace frees it); FWI calls are serialised.  Returns
 * HELM_OK, HELM_NOT_CONVERGED if any solve missed tol (outputs are still
 * written), HELM_ENAN if any solve produced a non-finite residual, or another
 * hard error.
 */
int fwi_misfit_grad(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                    const void* dobs, double tol, const helm_solve_opts* opt, double* misfit, float* grad,
                    int* iters, void* stream);

/*
 * fwi_misfit_grad_encoded -- the same misfit with simultaneous sources
 * (Sec. 3.2, eq. (3.6)-(3.8)): for an nsrc x p matrix X (Rademacher columns in
 * the method; any finite real matrix is accepted), the source sum of each
 * frequency is replaced by its trace estimate
 *   Phi_X = 1/2 (1/p) sum_f sum_i || R H_f^{-1} G x_i - D_f x_i ||^2,
 * G x_i = sum_s X[s][i] g_s and D_f x_i = sum_s X[s][i] d_fs, and grad is dPhi_X/dm.
 * Every receiver records every source, so the observed data are the data of the
 * encoded sum (the auxiliary data of eq. (3.7) coincide with them).
 *   X: float [nsrc][p] (host), drawn by the caller;
 *   dobs: the unencoded observed data, c64 [nfreq][nsrc][nrec] (device);
 *   iters (host, may be NULL): [2][nfreq][p];
 *   the other arguments as for fwi_misfit_grad.
 * nfreq * p forward and nfreq * p adjoint solves instead of nfreq * nsrc of
 * each.  X = the nsrc x nsrc identity gives fwi_misfit_grad's misfit and
 * gradient divided by nsrc.  Returns as fwi_misfit_grad; EINVAL for p <= 0 or a
 * non-finite entry of X.
 */
int fwi_misfit_grad_encoded(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const float* X, int p,
                            const int* rec_idx, int nrec, const void* dobs, double tol, const helm_solve_opts* opt,
                            double* misfit, float* grad, int* iters, void* stream);

/*
 * Linearised data (Gauss-Newton, eq. (3.9)-(3.11); the Jacobian's sign derived
 * from eq. (3.1)): with the point-source fields u_fs = H_f^{-1} g_s of the
 * operators' model m,
 *   fwi_born:          jdm = J dm,  J dm_fs = R H_f^{-1} (w_f^2 (1 - i gamma) u_fs dm),
 *                      dm float [nz][nx] (device) -> jdm c64 [nfreq][nsrc][nrec] (device);
 *   fwi_born_adjoint:  out = Re(J^H dd) = sum_fs w_f^2 Re(conj(lambda_fs) (1 - i gamma) u_fs),
 *                      lambda_fs = H_f^{-*} R^T dd_fs by conjugation (eq. (4.8)),
 *                      dd c64 [nfreq][nsrc][nrec] (device) -> out float [nz][nx] (device);
 *   fwi_gn_hessvec:    out = Re(J^H J dm), the Gauss-Newton Hessian of the misfit
 *                      applied to dm (what CG on the Gauss-Newton system needs).
 * Sources, receivers, tol and opt as for fwi_misfit_grad (every solve at tol).
 * iters (host, may be NULL) receives [nfreq][nsrc] per solve batch: forward
 * then Born (fwi_born), forward then adjoint (fwi_born_adjoint), forward, Born,
 * adjoint (fwi_gn_hessvec).  Each batch is one helm_solve call over all (f, s).
 * Workspace from the shared FWI pool.  Returns as fwi_misfit_grad.
 */
int fwi_born(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
             const float* dm, double tol, const helm_solve_opts* opt, void* jdm, int* iters, void* stream);
int fwi_born_adjoint(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                     const void* dd, double tol, const helm_solve_opts* opt, float* out, int* iters, void* stream);
int fwi_gn_hessvec(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                   const float* dm, double tol, const helm_solve_opts* opt, float* out, int* iters, void* stream);

/* Regularisers of the inversion's objective Phi(m) + alpha R(m) (Sec. 5):
 * with d = m - m_ref, grad_h the forward differences between neighbouring
 * nodes and Lap_h = -grad_h^T grad_h (each node sums (d_nb - d) / h^2 over the
 * neighbours that exist),
 *   FWI_REG_HIGH  R = ||Lap_h d||^2   (eq. (5.1), "spline smoothing"),
 *   FWI_REG_DIFF  R = ||grad_h d||^2  (eq. (5.2), diffusion);
 * sums over nodes and edges.  Gradients 2 Lap_h^2 d and -2 Lap_h d; Hessians
 * 2 Lap_h^2 and -2 Lap_h (the alpha nabla^2 R term of eq. (3.11)). */
#define FWI_REG_NONE 0
#define FWI_REG_HIGH 1
#define FWI_REG_DIFF 2

/* Options of the Gauss-Newton entry points. */
typedef struct {
    double damping;       /* >= 0: damping * I is added to the Gauss-Newton matrix    */
    int cg_iters;         /* conjugate-gradient steps (>= 0)                          */
    double tol_sens;      /* tolerance of the Born and adjoint solves inside CG
                             (Sec. 5.4 uses 1e-4); <= 0: the forward tol               */
    int reg;              /* FWI_REG_NONE / FWI_REG_HIGH / FWI_REG_DIFF               */
    double alpha;         /* weight of R (>= 0)                                       */
    const float* m_ref;   /* reference model, float [nz][nx] (device); needed when reg != NONE */
} fwi_gn_opts;

/*
 * fwi_gn_cg -- g->cg_iters conjugate-gradient steps from x = 0 on the
 * Gauss-Newton system (Re(J^H J) + alpha nabla^2 R + damping I) x = b, the
 * inner solve of a Gauss-Newton step (Sec. 3.3, eq. (3.9)-(3.11)), with the
 * products of fwi_gn_hessvec: the point-source fields are computed once (at
 * tol) and reused, and each step costs one Born and one adjoint solve batch
 * (at g->tol_sens).
 *   b, x: float [nz][nx] (device); the vector work (and the regulariser's
 *     Hessian) is FP64 and dot products are folded in a fixed order (same bits
 *     on every run);
 *   resnorms (host, may be NULL): [cg_iters + 1] norms ||b - A x_k||;
 *   iters (host, may be NULL): [cg_iters][2][nfreq][nsrc], the Born then the
 *     adjoint batch of each step (0 after an early stop);
 *   sources, receivers, tol and opt as for fwi_born.
 * Stops early, with the remaining norms 0, when the residual is exactly 0.
 * Returns as fwi_born, or HELM_ENAN if p.Ap <= 0 (a direction without
 * curvature, possible only without damping and regularisation).
 */
int fwi_gn_cg(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
              const float* b, const fwi_gn_opts* g, double tol, const helm_solve_opts* opt, float* x,
              double* resnorms, int* iters, void* stream);

/*
 * fwi_gn_step -- one Gauss-Newton step of the inversion (Sec. 3.3) on the
 * objective Phi(m) + alpha R(m): the data misfit and gradient at m (as
 * fwi_misfit_grad, at tol), plus alpha dR/dm; dm from g->cg_iters CG steps on
 * (Re(J^H J) + alpha nabla^2 R + damping I) dm = -grad (as fwi_gn_cg, the
 * sensitivities at g->tol_sens); m_new = m + mu dm.  One step of a window of
 * Alg. 1 (frequency continuation).
 *   m: float [nz][nx] (device), the model the operators were set up with
 *     (checked: HELM_EINVAL otherwise); m_new (device) may alias m;
 *   dobs: c64 [nfreq][nsrc][nrec] (device);
 *   misfit (host): the data misfit Phi(m); reg_value (host, may be NULL): R(m);
 *   grad (device, float [nz][nx]): dPhi/dm + alpha dR/dm at m;
 *   resnorms (host, may be NULL): [cg_iters + 1] CG residual norms;
 *   iters (host, may be NULL): [2 + 2 cg_iters][nfreq][nsrc]: the forward and
 *     adjoint batches of the gradient, then the Born and adjoint batches of
 *     each CG step.
 * The CG reuses the gradient's point-source fields: a step costs 2 + 2 cg_iters
 * solve batches.  Returns as fwi_gn_cg; EINVAL for a non-finite mu.
 */
int fwi_gn_step(const helm_op_t* ops, int nfreq, const int* src_idx, int nsrc, const int* rec_idx, int nrec,
                const void* dobs, const float* m, const fwi_gn_opts* g, double mu, double tol,
                const helm_solve_opts* opt, float* m_new, double* misfit, double* reg_value, float* grad,
                double* resnorms, int* iters, void* stream);

/* Frees the device workspace pool of the FWI entry points (the next call
 * allocates it again).  Synchronises the device. */
int fwi_release_workspace(void);

/*
 * helm_autotune -- kernel selection for the network's convolutions.  With
 * autotuning on (the default), the first eager launch of each convolution shape
 * times every applicable kernel (halo-tiled persistent with 16 or 32 output
 * channels / one tile per block with 32 or 64, implicit GEMM with 64x64, 128x32,
 * 64x128 or 128x64 tiles, the direct first-layer kernel) on the caller's
 * buffers and keeps the fastest for that shape for the rest of the process;
 * launches inside a stream capture use the built-in rule until the shape has
 * been tuned eagerly.  enable: 1 on, 0 off (built-in rule only), 2 forget the tuned
 * shapes, -1 leave unchanged.  tuned_shapes (host, may be NULL): number of
 * shapes tuned so far.
 */
int helm_autotune(int enable, int* tuned_shapes);
/* Tuned kernel choices to (save = 1) or from (save = 0, merged into the current
 * table) a text file (host path), so that another process launches exactly the
 * same kernels for the same shapes. */
int helm_autotune_file(const char* path, int save);
/* Diagnostics: pin the convolution kernel.  kernel in 0 .. kernel_count - 1 makes
 * every convolution launch for which that kernel applies use it (bypassing the
 * autotuner and the built-in rule; launches it does not apply to keep their
 * usual choice); -1 removes the pin.  kernel_count (host, may be NULL) receives
 * the number of kernel kinds.  For tests that check each kernel against a
 * reference; EINVAL for an id outside -1 .. kernel_count - 1. */
int helm_conv_force(int kernel, int* kernel_count);

/*
 * Diagnostics: time the launches of one named kernel family ("k_matvec_dot",
 * "k_update", "k_mg_down", "k_mg_up", "k_poly_lds", "k_conv", ...) with
 * fence-free HIP events recorded on the stream each is launched on, and count
 * the algorithmic bytes (or flops) their active blocks processed.  Launches
 * recorded into a stream capture are neither timed nor counted (a replayed
 * graph has no per-launch events).  kernel = NULL stops timing.
 * helm_ktimer_sample(every) samples on average one launch in every of the
 * family (the first after helm_ktimer_start, then by a fixed hash of the launch
 * index, so that no layer of a repeated sequence is favoured; default 1 = all),
 * which keeps the event packets from slowing a long run; time and work are then
 * both taken over the sampled launches.  helm_ktimer_read synchronises the device and
 * returns the sampled launches, their total event time and their total work
 * since the last start (host outputs).
 */
int helm_ktimer_start(const char* kernel);
int helm_ktimer_sample(int every);
/* Sample whole restart cycles of helm_solve instead: every launch of the
 * family inside one in every cycles (by the same hash of the cycle index) is
 * timed and counted, on whichever stream it runs. */
int helm_ktimer_sample_steps(int every);
int helm_ktimer_read(int* launches, double* total_ms, double* total_work);
/* All eager launches of the named family since helm_ktimer_start, sampled or
 * not (host output). */
int helm_ktimer_count(long long* launches);
/* Length of the union of the sampled launches' [start, end] intervals since
 * helm_ktimer_start, in ms (host output; synchronises the device).  Without
 * overlap it equals helm_ktimer_read's total; when the family's launches run
 * concurrently on several streams, with every = 1 it is the wall time during
 * which at least one of them ran. */
int helm_ktimer_busy(double* busy_ms);

const char* helm_last_error(void);
/* Library version string. */
const char* helm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
