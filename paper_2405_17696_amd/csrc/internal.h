// Internal structures shared by the translation units of libhelm.
#pragma once
#include <vector>

#include "common.h"

struct cnn_net;

namespace helm {

constexpr int MAX_LEVELS = 4;
constexpr int PAIRS_PER_BLOCK = 512;  // level-0 vector kernels: 256 threads x 2 node pairs
constexpr int VEC_THREADS = 256;
constexpr int MAX_RESTART = 64;
constexpr uint32_t COARSE_KEY0 = 0x48454C4Du, COARSE_KEY1 = 0x5F534C31u;

// Second-difference coefficients of one level.  The far boundary lies a
// distance delta beyond the last row/column; there the stencil is
// 2/(H+delta) [(1/delta + 1/H) u - u_W / H] (regular when delta = H).
template <typename T>
struct Sten {
    T ax, az;    // 1/H^2: neighbour coefficients in the interior
    T axl, dxl;  // last column: west coefficient, x part of the diagonal
    T azl, dzl;  // last row: north coefficient, z part of the diagonal
};

struct Level {
    int nz = 0, nx = 0;
    double hx = 0, hz = 0;
    double dx = 0, dz = 0;  // distance from the last column / row to the far boundary
    template <typename T>
    Sten<T> sten() const {
        Sten<T> s;
        s.ax = T(1.0 / (hx * hx));
        s.az = T(1.0 / (hz * hz));
        s.axl = T(2.0 / ((hx + dx) * hx));
        s.dxl = T(2.0 / (hx + dx) * (1.0 / dx + 1.0 / hx));
        s.azl = T(2.0 / ((hz + dz) * hz));
        s.dzl = T(2.0 / (hz + dz) * (1.0 / dz + 1.0 / hz));
        return s;
    }
    float* k2 = nullptr;   // restricted squared slowness (level 0: the input copy)
    float* g = nullptr;    // restricted attenuation
    c64* sl32 = nullptr;   // shifted-Laplacian mass term omega^2 m (1 - (g + beta) i)
    c128* sl64 = nullptr;
    c64* wd32 = nullptr;   // damped-Jacobi factor w / D, D = diagonal of the level operator
    c128* wd64 = nullptr;
    long n() const { return (long)nz * nx; }
};

// Encoder context of one (network, operator) pair.
struct EncCache {
    const cnn_net* net = nullptr;
    uint64_t net_version = 0;
    void* ctx = nullptr;   // owned by the CNN module
};

}  // namespace helm

struct helm_op {
    int nz = 0, nx = 0;
    double hx = 0, hz = 0, omega = 0, beta = 0.5, jw = 0.8;
    int with_gamma = 1;
    int nlev = 3;
    int degree = 20;
    helm::c64* coef32 = nullptr;   // omega^2 m (1 - i gamma)
    helm::c128* coef64 = nullptr;
    helm::Level lv[helm::MAX_LEVELS];
    std::vector<helm::c128> roots;  // coarsest-level polynomial roots, Leja order
    helm::c128* roots_dev = nullptr;
    bool poly_lds_ok = false;
    helm::EncCache enc;
    long n() const { return (long)nz * nx; }
};

namespace helm {

// Per-RHS Krylov state, device resident.
struct RhsState {
    double bnorm;
    double relres;   // last FP64 true relative residual
    double est;      // Givens estimate |g_{j+1}| / ||b||
    double wb2;      // ||w||^2 before orthogonalisation (current step)
    int active;      // iterating in the current cycle
    int cycdone;     // current cycle finished early
    int jlen;        // Arnoldi steps done in the current cycle
    int iters;       // total Arnoldi steps
    int status;      // HELM_OK / HELM_NOT_CONVERGED / HELM_ENAN
    int need2;       // second Gram-Schmidt pass requested for this step
    int done;        // solve finished
    int cycles;
    int maxit;       // iteration cap of this RHS
};

// One group of right-hand sides sharing an operator.
template <typename T>
struct GroupArgs {
    int nz, nx, nblk, rhs0;
    long N, off0;
    T ax, az;                  // 1/hx^2, 1/hz^2
    const cx<T>* coef;         // omega^2 m (1 - i gamma) in precision T
    const float* k2;           // for the FP64 residual
    const float* gam;
    double omega2, axd, azd;
};

// Global solve arguments.
template <typename T>
struct SolveArgs {
    int m, nrhs, maxblk, maxit, conjop, reorth;
    long Ntot;
    double tol;
    cx<T>* V;        // [m+1][Ntot]
    cx<T>* Z;        // [m][Ntot]
    const c64* b;    // [Ntot]
    c128* x;         // [Ntot]
    RhsState* st;    // [nrhs]
    c128* H;         // [nrhs][m][m+1]  column j at H + (r*m + j)*(m+1)
    c128* cs;        // [nrhs][m]
    c128* sn;        // [nrhs][m]
    c128* g;         // [nrhs][m+1]
    double* vscale;  // [nrhs][m+1]
    c128* hcur;      // [nrhs][m+1]
    c128* y;         // [nrhs][m]
    c128* part;      // [nrhs][maxblk][m+2]
};

// ---------------------------------------------------------------- launchers (helm_kernels.hip)
template <typename T>
int launch_matvec(const helm_op* op, const cx<T>* u, cx<T>* v, int nrhs, int conj, hipStream_t s);

int setup_levels(helm_op* op, const float* k2, const float* g, hipStream_t s);

// V-cycle on a group: f (scaled per RHS by fscale[r*fstride] when fscale != nullptr)
// -> out (+ addend when addend != nullptr).  st masks inactive RHS (may be null).
template <typename T>
struct MgWork {
    cx<T>* f[MAX_LEVELS];   // level >= 1 right-hand sides
    cx<T>* e[MAX_LEVELS];   // level >= 1 corrections (coarsest: polynomial iterate)
    c128* ra;               // coarsest-level polynomial residual ping-pong (FP64)
    c128* rb;
    c128* xw;               // coarsest-level polynomial iterate (FP64)
};
template <typename T>
int launch_vcycle(const helm_op* op, const cx<T>* f, const double* fscale, int fstride, cx<T>* out,
                  const cx<T>* addend, int nrhs, const RhsState* st, int rhs0, MgWork<T>& w, hipStream_t s);

template <typename T>
size_t mg_work_elems(const helm_op* op, int level);

template <typename T>
void fill_group(GroupArgs<T>& g, const helm_op* op, int rhs0, long off0);

// Krylov kernels
template <typename T>
int launch_true_residual(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, hipStream_t s);
template <typename T>
int launch_matvec_dot(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s);
template <typename T>
int launch_update(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, int pass, hipStream_t s);
template <typename T>
int launch_dot2(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s);
template <typename T>
int launch_lsq(const SolveArgs<T>& a, hipStream_t s);
template <typename T>
int launch_sol_update(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, hipStream_t s);
template <typename T>
int launch_scale_copy(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, hipStream_t s);
template <typename T>
int launch_residual_vs_e0(const GroupArgs<T>& g, int ng, const SolveArgs<T>& a, int j, const cx<T>* e0,
                          cx<T>* out, hipStream_t s);
int launch_init_state(RhsState* st, int nrhs, const int* maxit_rhs, int maxit, hipStream_t s);
int launch_zero_done_x(const GroupArgs<double>& g, int ng, const RhsState* st, c128* x, hipStream_t s);

// Fixed-iteration, MG-preconditioned GMRES used by the training-data generation
// (eq. 4.3) and the light-weight retraining: exactly iters[r] (host) Arnoldi steps
// for RHS r from x (x0_given) or zero; rhs c64, x c128, one operator.
int solve_fixed_iters(const helm_op* op, const c64* rhs, c128* x, int nrhs, const int* iters, int x0_given,
                      hipStream_t s);

// host linear algebra (hostla.cpp)
std::vector<c128> hessenberg_eigvals(std::vector<c128> A, int n);
std::vector<c128> leja_order(const std::vector<c128>& th);
std::vector<c128> coarse_roots_host(const Level& L, int degree);

}  // namespace helm
