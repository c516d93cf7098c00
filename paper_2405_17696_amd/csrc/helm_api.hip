// C ABI of libhelm: operator handles, matvec, V-cycle, and the batched
// flexible-GMRES driver (host side; the kernels live in helm_kernels.hip).
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "cnn.h"
#include "internal.h"

namespace helm {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return HELM_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t b = std::max<size_t>(bytes, 256);
        if (hipMalloc(&p, b) != hipSuccess) return fail(HELM_ENOMEM, "hipMalloc(%zu) failed", b);
        cap = b;
        return HELM_OK;
    }
};

template <typename T>
static int alloc(T** p, size_t n) {
    if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
        return fail(HELM_ENOMEM, "hipMalloc(%zu) failed", n * sizeof(T));
    return HELM_OK;
}

// ------------------------------------------------------------------ conj kernels
template <typename T>
__global__ void k_conj_copy(const cx<T>* __restrict__ a, cx<T>* __restrict__ b, long n) {
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = conj(a[t]);
}

// Bilinear resampling of a nodal field onto an mz x mx grid of the same extent
// (output node (I, K) sits at input coordinates I (nz-1)/(mz-1), K (nx-1)/(mx-1)).
__global__ void k_resample(const float* __restrict__ in, int nz, int nx, float* __restrict__ out, int mz, int mx) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)mz * mx) return;
    const int I = (int)(t / mx), K = (int)(t - (long)I * mx);
    const double z = mz > 1 ? (double)I * (nz - 1) / (mz - 1) : 0.0;
    const double x = mx > 1 ? (double)K * (nx - 1) / (mx - 1) : 0.0;
    int i0 = (int)z, k0 = (int)x;
    if (i0 > nz - 2) i0 = nz > 1 ? nz - 2 : 0;
    if (k0 > nx - 2) k0 = nx > 1 ? nx - 2 : 0;
    const double a = nz > 1 ? z - i0 : 0.0, b = nx > 1 ? x - k0 : 0.0;
    const int i1 = nz > 1 ? i0 + 1 : i0, k1 = nx > 1 ? k0 + 1 : k0;
    const double v = (1 - a) * ((1 - b) * in[(long)i0 * nx + k0] + b * in[(long)i0 * nx + k1]) +
                     a * ((1 - b) * in[(long)i1 * nx + k0] + b * in[(long)i1 * nx + k1]);
    out[t] = (float)v;
}

template <typename T>
static int conj_copy(const cx<T>* a, cx<T>* b, long n, hipStream_t s) {
    if (n == 0) return HELM_OK;
    hipLaunchKernelGGL(k_conj_copy<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

// ------------------------------------------------------------------ solve workspace
struct SolveWork {
    DevBuf V, Z, st, H, cs, sn, g, vscale, hcur, y, part, bconj, maxit;
    DevBuf mg[2 * MAX_LEVELS + 3];
    DevBuf cnn_e0, cnn_res;
    std::vector<RhsState> hst;
};
static SolveWork g_work;
static std::mutex g_mutex;

struct GraphHolder {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphHolder() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Streams cannot be captured when they are the legacy default stream; graph
// replays then run on a library stream ordered after the caller's stream.
static hipStream_t graph_stream() {
    static hipStream_t gs = nullptr;
    if (!gs) (void)hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
    return gs;
}

// Second stream of a preconditioner step split in two halves, with the events
// that fork it from and join it back to the solve's stream.
struct SplitStream {
    hipStream_t s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
static int split_stream(SplitStream** out) {
    static SplitStream ss;
    if (!ss.s2 && (hipStreamCreateWithFlags(&ss.s2, hipStreamNonBlocking) != hipSuccess ||
                   hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) != hipSuccess ||
                   hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) != hipSuccess)) {
        ss.s2 = nullptr;
        return fail(HELM_EHIP, "helm_solve: second stream");
    }
    *out = &ss;
    return HELM_OK;
}

// The multigrid scratch of a batch, seen from its RHS `first` on.
template <typename T>
static MgWork<T> mg_from(const MgWork<T>& w, const helm_op* op, int first) {
    MgWork<T> v = w;
    for (int l = 1; l < op->nlev; ++l) {
        v.f[l] += (long)first * op->lv[l].n();
        v.e[l] += (long)first * op->lv[l].n();
    }
    const long nc = (long)first * op->lv[op->nlev - 1].n();
    v.ra += nc;
    v.rb += nc;
    v.xw += nc;
    return v;
}

template <typename T>
static int solve_impl(const helm_op_t* ops, int nops, const int* rhs_op, const void* rhs, void* xv, int nrhs,
                      double tol, const helm_solve_opts& o, int* iters, double* relres, int* status, hipStream_t s,
                      const int* maxit_rhs_host = nullptr) {
    SolveWork& W = g_work;
    // groups of consecutive RHS sharing an operator
    struct Grp {
        int op, r0, n;
        long off0;
    };
    std::vector<Grp> groups;
    long Ntot = 0;
    int maxblk = 1;
    for (int r = 0; r < nrhs; ++r) {
        int k = rhs_op ? rhs_op[r] : 0;
        if (k < 0 || k >= nops) return fail(HELM_EINVAL, "rhs_op[%d] = %d out of range", r, k);
        if (!groups.empty() && groups.back().op == k) {
            groups.back().n++;
        } else {
            for (auto& gg : groups)
                if (gg.op == k) return fail(HELM_EINVAL, "rhs_op must group RHS by operator (index %d)", r);
            groups.push_back({k, r, 1, Ntot});
        }
        Ntot += ops[k]->n();
        int nb = (int)((ops[k]->n() / 2 + PAIRS_PER_BLOCK - 1) / PAIRS_PER_BLOCK);
        maxblk = std::max(maxblk, nb);
    }
    const int m = o.restart;
    const int K = m + 2;
    int rc;
    if ((rc = W.V.ensure(sizeof(cx<T>) * (size_t)(m + 1) * Ntot))) return rc;
    if ((rc = W.Z.ensure(sizeof(cx<T>) * (size_t)m * Ntot))) return rc;
    if ((rc = W.st.ensure(sizeof(RhsState) * nrhs))) return rc;
    if ((rc = W.H.ensure(sizeof(c128) * (size_t)nrhs * m * (m + 1)))) return rc;
    if ((rc = W.cs.ensure(sizeof(c128) * (size_t)nrhs * m))) return rc;
    if ((rc = W.sn.ensure(sizeof(c128) * (size_t)nrhs * m))) return rc;
    if ((rc = W.g.ensure(sizeof(c128) * (size_t)nrhs * (m + 1)))) return rc;
    if ((rc = W.vscale.ensure(sizeof(double) * (size_t)nrhs * (m + 1)))) return rc;
    if ((rc = W.hcur.ensure(sizeof(c128) * (size_t)nrhs * (m + 1)))) return rc;
    if ((rc = W.y.ensure(sizeof(c128) * (size_t)nrhs * m))) return rc;
    if ((rc = W.part.ensure(sizeof(c128) * (size_t)nrhs * maxblk * K))) return rc;
    // multigrid scratch, reused group after group
    const bool use_mg = o.precond == HELM_PRECOND_MG || o.precond == HELM_PRECOND_CNN_VU;
    const bool use_cnn = o.precond == HELM_PRECOND_CNN || o.precond == HELM_PRECOND_CNN_VU;
    const bool two_streams = use_cnn && o.streams == 2;
    SplitStream* sp = nullptr;
    if (two_streams && (rc = split_stream(&sp))) return rc;
    std::vector<MgWork<T>> mgw(groups.size());
    if (use_mg) {
        size_t need[MAX_LEVELS] = {0};
        size_t needc = 0;
        for (auto& gr : groups) {
            const helm_op* op = ops[gr.op];
            for (int l = 1; l < op->nlev; ++l) need[l] = std::max(need[l], (size_t)gr.n * op->lv[l].n());
            needc = std::max(needc, (size_t)gr.n * op->lv[op->nlev - 1].n());
        }
        for (int l = 1; l < MAX_LEVELS; ++l) {
            if ((rc = W.mg[2 * l].ensure(sizeof(cx<T>) * need[l]))) return rc;
            if ((rc = W.mg[2 * l + 1].ensure(sizeof(cx<T>) * need[l]))) return rc;
        }
        for (int q = 0; q < 3; ++q)
            if ((rc = W.mg[2 * MAX_LEVELS + q].ensure(sizeof(c128) * needc))) return rc;
        for (auto& w : mgw) {
            for (int l = 0; l < MAX_LEVELS; ++l) {
                w.f[l] = (cx<T>*)W.mg[2 * l].p;
                w.e[l] = (cx<T>*)W.mg[2 * l + 1].p;
            }
            w.ra = (c128*)W.mg[2 * MAX_LEVELS].p;
            w.rb = (c128*)W.mg[2 * MAX_LEVELS + 1].p;
            w.xw = (c128*)W.mg[2 * MAX_LEVELS + 2].p;
        }
    }
    if (use_cnn) {
        size_t maxg = 0;
        for (auto& gr : groups) maxg = std::max(maxg, (size_t)gr.n * ops[gr.op]->n());
        if ((rc = W.cnn_e0.ensure(sizeof(cx<T>) * maxg))) return rc;
        if ((rc = W.cnn_res.ensure(sizeof(cx<T>) * maxg))) return rc;
        for (auto& gr : groups) {
            if (two_streams && gr.n >= 2) {
                const int na = (gr.n + 1) / 2;
                if ((rc = cnn_prepare(o.net, ops[gr.op], na, s, 0))) return rc;
                if ((rc = cnn_prepare(o.net, ops[gr.op], gr.n - na, s, 1))) return rc;
            } else if ((rc = cnn_prepare(o.net, ops[gr.op], gr.n, s))) {
                return rc;
            }
        }
    }

    const c64* b = (const c64*)rhs;
    c128* x = (c128*)xv;
    if (o.adjoint) {
        // H^* x = b  <=>  H conj(x) = conj(b)   (eq. (4.8))
        if ((rc = W.bconj.ensure(sizeof(c64) * Ntot))) return rc;
        if ((rc = conj_copy<float>(b, (c64*)W.bconj.p, Ntot, s))) return rc;
        b = (const c64*)W.bconj.p;
        if (o.x0_given && (rc = conj_copy<double>(x, x, Ntot, s))) return rc;
    }
    if (!o.x0_given) HELM_HIP(hipMemsetAsync(x, 0, sizeof(c128) * Ntot, s));
    HELM_HIP(hipMemsetAsync(W.st.p, 0, sizeof(RhsState) * nrhs, s));
    const int* maxit_dev = nullptr;
    if (maxit_rhs_host) {
        if ((rc = W.maxit.ensure(sizeof(int) * nrhs))) return rc;
        HELM_HIP(hipMemcpyAsync(W.maxit.p, maxit_rhs_host, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        maxit_dev = (const int*)W.maxit.p;
    }
    if ((rc = launch_init_state((RhsState*)W.st.p, nrhs, maxit_dev, o.maxit, s))) return rc;

    SolveArgs<T> a;
    a.m = m;
    a.nrhs = nrhs;
    a.maxblk = maxblk;
    a.maxit = o.maxit;
    a.conjop = 0;
    a.reorth = o.reorth;
    a.Ntot = Ntot;
    a.tol = tol;
    a.V = (cx<T>*)W.V.p;
    a.Z = (cx<T>*)W.Z.p;
    a.b = b;
    a.x = x;
    a.st = (RhsState*)W.st.p;
    a.H = (c128*)W.H.p;
    a.cs = (c128*)W.cs.p;
    a.sn = (c128*)W.sn.p;
    a.g = (c128*)W.g.p;
    a.vscale = (double*)W.vscale.p;
    a.hcur = (c128*)W.hcur.p;
    a.y = (c128*)W.y.p;
    a.part = (c128*)W.part.p;

    std::vector<GroupArgs<T>> ga(groups.size());
    std::vector<GroupArgs<double>> gd(groups.size());
    for (size_t i = 0; i < groups.size(); ++i) {
        fill_group<T>(ga[i], ops[groups[i].op], groups[i].r0, groups[i].off0);
        fill_group<double>(gd[i], ops[groups[i].op], groups[i].r0, groups[i].off0);
    }
    W.hst.resize(nrhs);

    // A CNN preconditioner on RHS first .. first + nh - 1 of group gi (its network
    // workspaces: slot), on stream sh.  M_VU: e0 = M_net(v), then the V-cycle of
    // the residual v - H e0 added to e0; a right-hand side whose network output is
    // not finite gets e0 = 0, i.e. M_VU = V_SL for that step.
    auto precond_part = [&](size_t gi, int first, int nh, int j, hipStream_t sh, int slot) -> int {
        const Grp& gr = groups[gi];
        const helm_op* op = ops[gr.op];
        const long so = (long)first * op->n();
        cx<T>* vj = a.V + (long)j * Ntot + gr.off0 + so;
        cx<T>* zj = a.Z + (long)j * Ntot + gr.off0 + so;
        if (o.precond == HELM_PRECOND_CNN)
            return cnn_apply_masked(o.net, op, (const void*)vj, a.vscale + j, m + 1, (void*)zj, nh, a.st,
                                    gr.r0 + first, sizeof(T) == 8, sh, false, slot);
        cx<T>* e0 = (cx<T>*)W.cnn_e0.p + so;
        cx<T>* res = (cx<T>*)W.cnn_res.p + so;
        GroupArgs<T> gh = ga[gi];
        gh.rhs0 += first;
        gh.off0 += so;
        MgWork<T> wh = mg_from(mgw[gi], op, first);
        int r = cnn_apply_masked(o.net, op, (const void*)vj, a.vscale + j, m + 1, (void*)e0, nh, a.st, gr.r0 + first,
                                 sizeof(T) == 8, sh, true, slot);
        if (!r) r = launch_residual_vs_e0<T>(gh, nh, a, j, e0, res, sh);
        if (!r) r = launch_vcycle<T>(op, res, nullptr, 0, zj, e0, nh, a.st, gr.r0 + first, wh, sh);
        return r;
    };

    auto precond = [&](int j) -> int {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Grp& gr = groups[gi];
            const helm_op* op = ops[gr.op];
            cx<T>* vj = a.V + (long)j * Ntot + gr.off0;
            cx<T>* zj = a.Z + (long)j * Ntot + gr.off0;
            int r;
            switch (o.precond) {
                case HELM_PRECOND_NONE:
                    r = launch_scale_copy<T>(ga[gi], gr.n, a, j, s);
                    break;
                case HELM_PRECOND_MG:
                    r = launch_vcycle<T>(op, vj, a.vscale + j, m + 1, zj, nullptr, gr.n, a.st, gr.r0, mgw[gi], s);
                    break;
                case HELM_PRECOND_CNN:
                case HELM_PRECOND_CNN_VU:
                    if (two_streams && gr.n >= 2) {
                        // the two halves of the group on two streams, each on its own workspaces,
                        // joined before the Arnoldi step (and before the next group, which reuses
                        // the scratch)
                        const int na = (gr.n + 1) / 2;
                        HELM_HIP(hipEventRecord(sp->fork, s));
                        HELM_HIP(hipStreamWaitEvent(sp->s2, sp->fork, 0));
                        r = precond_part(gi, 0, na, j, s, 0);
                        if (!r) r = precond_part(gi, na, gr.n - na, j, sp->s2, 1);
                        HELM_HIP(hipEventRecord(sp->join, sp->s2));
                        HELM_HIP(hipStreamWaitEvent(s, sp->join, 0));
                    } else {
                        r = precond_part(gi, 0, gr.n, j, s, 0);
                    }
                    break;
                default:
                    return fail(HELM_EINVAL, "unknown preconditioner %d", o.precond);
            }
            if (r) return r;
        }
        return HELM_OK;
    };

    // One restart cycle (Arnoldi steps, least squares, update of x) followed
    // by the true residual that opens the next cycle.  Eager, or replayed
    // from a graph captured on the first cycle.
    auto cycle_body = [&]() -> int {
        int r = HELM_OK;
        ktimer().step(s);
        for (int j = 0; j < m; ++j) {
            if ((r = precond(j))) return r;
            for (size_t gi = 0; gi < groups.size(); ++gi)
                if ((r = launch_matvec_dot<T>(ga[gi], groups[gi].n, a, j, s))) return r;
            for (size_t gi = 0; gi < groups.size(); ++gi)
                if ((r = launch_update<T>(ga[gi], groups[gi].n, a, j, 1, s))) return r;
            if (o.reorth) {
                for (size_t gi = 0; gi < groups.size(); ++gi)
                    if ((r = launch_dot2<T>(ga[gi], groups[gi].n, a, j, s))) return r;
                for (size_t gi = 0; gi < groups.size(); ++gi)
                    if ((r = launch_update<T>(ga[gi], groups[gi].n, a, j, 2, s))) return r;
            }
        }
        if ((r = launch_lsq<T>(a, s))) return r;
        for (size_t gi = 0; gi < groups.size(); ++gi)
            if ((r = launch_sol_update<T>(ga[gi], groups[gi].n, a, s))) return r;
        for (size_t gi = 0; gi < groups.size(); ++gi)
            if ((r = launch_true_residual<T>(ga[gi], groups[gi].n, a, s))) return r;
        return HELM_OK;
    };

    for (size_t gi = 0; gi < groups.size(); ++gi)
        if ((rc = launch_true_residual<T>(ga[gi], groups[gi].n, a, s))) return rc;
    for (size_t gi = 0; gi < groups.size(); ++gi)
        if ((rc = launch_zero_done_x(gd[gi], groups[gi].n, a.st, x, s))) return rc;
    GraphHolder gh;
    const int max_cycles = o.maxit + 2;
    for (int cyc = 0; cyc <= max_cycles; ++cyc) {
        HELM_HIP(hipMemcpyAsync(W.hst.data(), a.st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, s));
        HELM_HIP(hipStreamSynchronize(s));
        ktimer().harvest();
        int nact = 0;
        for (int r = 0; r < nrhs; ++r) nact += W.hst[r].active;
        if (nact == 0) break;
        if (o.use_graph) {
            if (!gh.exec) {
                ktimer().new_capture();
                HELM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                int r = cycle_body();
                hipError_t ce = hipStreamEndCapture(s, &gh.graph);
                if (r) return r;
                if (ce != hipSuccess) return fail(HELM_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
                HELM_HIP(hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0));
            }
            HELM_HIP(hipGraphLaunch(gh.exec, s));
            ktimer().replayed();
        } else if ((rc = cycle_body())) {
            return rc;
        }
    }
    if (o.adjoint && (rc = conj_copy<double>(x, x, Ntot, s))) return rc;
    HELM_HIP(hipStreamSynchronize(s));
    int worst = HELM_OK;
    for (int r = 0; r < nrhs; ++r) {
        const RhsState& S = W.hst[r];
        int stt = S.done ? S.status : HELM_NOT_CONVERGED;
        if (iters) iters[r] = S.iters;
        if (relres) relres[r] = S.relres;
        if (status) status[r] = stt;
        if (stt == HELM_NOT_CONVERGED && worst == HELM_OK) worst = HELM_NOT_CONVERGED;
        if (stt == HELM_ENAN) worst = HELM_NOT_CONVERGED;
    }
    return worst;
}

int solve_fixed_iters(const helm_op* op, const c64* rhs, c128* x, int nrhs, const int* iters, int x0_given,
                      hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mutex);
    helm_solve_opts o;
    memset(&o, 0, sizeof(o));
    o.precond = HELM_PRECOND_MG;
    int mx = 1;
    for (int r = 0; r < nrhs; ++r) mx = std::max(mx, iters[r]);
    o.restart = std::min(mx, MAX_RESTART);
    o.maxit = mx;
    o.x0_given = x0_given;
    helm_op_t ops[1] = {const_cast<helm_op*>(op)};
    std::vector<int> ro(nrhs, 0);
    int rc = solve_impl<float>(ops, 1, ro.data(), rhs, x, nrhs, 1e-300, o, nullptr, nullptr, nullptr, s, iters);
    return rc == HELM_NOT_CONVERGED ? HELM_OK : rc;
}

}  // namespace helm

using namespace helm;

extern "C" {

const char* helm_last_error(void) { return helm::g_err; }
const char* helm_version(void) { return "libhelm 0.1 (gfx950)"; }

int helm_setup(const float* kappa2, const float* gamma, int nz, int nx, double omega, double h,
               const helm_setup_opts* opt, void* stream, helm_op_t* out) {
    if (!out) return fail(HELM_EINVAL, "helm_setup: out is NULL");
    *out = nullptr;
    if (!kappa2 || !gamma) return fail(HELM_EINVAL, "helm_setup: NULL kappa2/gamma");
    if (nz < 4 || nx < 4 || (nx & 1)) return fail(HELM_EINVAL, "helm_setup: need nz, nx >= 4 and even nx (%d x %d)", nz, nx);
    if (!(h > 0) || !(omega > 0)) return fail(HELM_EINVAL, "helm_setup: h and omega must be positive");
    hipStream_t s = (hipStream_t)stream;
    helm_op* op = new helm_op();
    op->nz = nz;
    op->nx = nx;
    op->hx = h;
    op->hz = (opt && opt->hz > 0) ? opt->hz : h;
    op->omega = omega;
    op->beta = (opt && opt->sl_beta > 0) ? opt->sl_beta : 0.5;
    op->with_gamma = (opt && opt->sl_no_gamma) ? 0 : 1;
    op->nlev = (opt && opt->mg_levels > 0) ? opt->mg_levels : 3;
    op->degree = (opt && opt->coarse_degree > 0) ? opt->coarse_degree : 20;
    op->jw = (opt && opt->jacobi_weight > 0) ? opt->jacobi_weight : 0.8;
    if (op->nlev > MAX_LEVELS) {
        delete op;
        return fail(HELM_EINVAL, "helm_setup: mg_levels must be <= %d", MAX_LEVELS);
    }
    if (op->degree > 64) {
        delete op;
        return fail(HELM_EINVAL, "helm_setup: coarse_degree must be <= 64");
    }
    int rc = HELM_OK;
    int cz = nz, cxn = nx;
    for (int l = 0; l < op->nlev; ++l) {
        Level& L = op->lv[l];
        L.nz = cz;
        L.nx = cxn;
        L.hx = op->hx * (1 << l);
        L.hz = op->hz * (1 << l);
        // last node of level l sits on finest node 2^l * n_l - 1; the far boundary is at node n
        L.dz = (nz - ((1 << l) * L.nz - 1)) * op->hz;
        L.dx = (nx - ((1 << l) * L.nx - 1)) * op->hx;
        if (L.nz < 2 || L.nx < 2) {
            helm_destroy(op);
            return fail(HELM_EINVAL, "helm_setup: grid too small for %d levels", op->nlev);
        }
        long n = L.n();
        if ((rc = alloc(&L.k2, n)) || (rc = alloc(&L.g, n)) || (rc = alloc(&L.sl32, n)) || (rc = alloc(&L.sl64, n)) ||
            (rc = alloc(&L.wd32, n)) || (rc = alloc(&L.wd64, n))) {
            helm_destroy(op);
            return rc;
        }
        cz = cz / 2;
        cxn = cxn / 2;
    }
    long n = op->n();
    if ((rc = alloc(&op->coef32, n)) || (rc = alloc(&op->coef64, n))) {
        helm_destroy(op);
        return rc;
    }
    if (hipMemcpyAsync(op->lv[0].k2, kappa2, n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(op->lv[0].g, gamma, n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess) {
        helm_destroy(op);
        return fail(HELM_EHIP, "helm_setup: copy of kappa2/gamma failed");
    }
    if ((rc = setup_levels(op, kappa2, gamma, s))) {
        helm_destroy(op);
        return rc;
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        helm_destroy(op);
        return fail(HELM_EHIP, "helm_setup: stream synchronize failed");
    }
    op->roots = coarse_roots_host(op->lv[op->nlev - 1], op->degree);
    if ((int)op->roots.size() == 0) {
        helm_destroy(op);
        return fail(HELM_EHIP, "helm_setup: coarse polynomial failed");
    }
    if ((rc = alloc(&op->roots_dev, op->roots.size())) ||
        hipMemcpy(op->roots_dev, op->roots.data(), op->roots.size() * sizeof(c128), hipMemcpyHostToDevice) !=
            hipSuccess) {
        helm_destroy(op);
        return rc ? rc : fail(HELM_EHIP, "helm_setup: roots upload failed");
    }
    *out = op;
    return HELM_OK;
}

void helm_destroy(helm_op_t op) {
    if (!op) return;
    cnn_release_cache(op);
    for (int l = 0; l < MAX_LEVELS; ++l) {
        Level& L = op->lv[l];
        if (L.k2) (void)hipFree(L.k2);
        if (L.g) (void)hipFree(L.g);
        if (L.sl32) (void)hipFree(L.sl32);
        if (L.sl64) (void)hipFree(L.sl64);
        if (L.wd32) (void)hipFree(L.wd32);
        if (L.wd64) (void)hipFree(L.wd64);
    }
    if (op->roots_dev) (void)hipFree(op->roots_dev);
    if (op->coef32) (void)hipFree(op->coef32);
    if (op->coef64) (void)hipFree(op->coef64);
    delete op;
}

int helm_op_info(helm_op_t op, int* nz, int* nx, double* omega, double* hx, double* hz) {
    if (!op) return fail(HELM_EINVAL, "helm_op_info: NULL op");
    if (nz) *nz = op->nz;
    if (nx) *nx = op->nx;
    if (omega) *omega = op->omega;
    if (hx) *hx = op->hx;
    if (hz) *hz = op->hz;
    return HELM_OK;
}

int helm_matvec(helm_op_t op, const void* u, void* v, int nrhs, int dtype, int adjoint, void* stream) {
    if (!op || nrhs < 0) return fail(HELM_EINVAL, "helm_matvec: bad arguments");
    if (nrhs == 0) return HELM_OK;   // an empty batch: the buffers may be NULL
    if (!u || !v) return fail(HELM_EINVAL, "helm_matvec: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == HELM_C64) return launch_matvec<float>(op, (const c64*)u, (c64*)v, nrhs, adjoint, s);
    if (dtype == HELM_C128) return launch_matvec<double>(op, (const c128*)u, (c128*)v, nrhs, adjoint, s);
    return fail(HELM_EINVAL, "helm_matvec: dtype %d", dtype);
}

int helm_vcycle(helm_op_t op, const void* f, void* e, int nrhs, void* stream) {
    if (!op || nrhs < 0) return fail(HELM_EINVAL, "helm_vcycle: bad arguments");
    if (nrhs == 0) return HELM_OK;   // an empty batch: the buffers may be NULL
    if (!f || !e) return fail(HELM_EINVAL, "helm_vcycle: NULL buffer");
    std::lock_guard<std::mutex> lk(g_mutex);
    hipStream_t s = (hipStream_t)stream;
    SolveWork& W = g_work;
    MgWork<float> w;
    int rc;
    for (int l = 1; l < op->nlev; ++l) {
        if ((rc = W.mg[2 * l].ensure(sizeof(c64) * (size_t)nrhs * op->lv[l].n()))) return rc;
        if ((rc = W.mg[2 * l + 1].ensure(sizeof(c64) * (size_t)nrhs * op->lv[l].n()))) return rc;
    }
    size_t nc = (size_t)nrhs * op->lv[op->nlev - 1].n();
    for (int q = 0; q < 3; ++q)
        if ((rc = W.mg[2 * MAX_LEVELS + q].ensure(sizeof(c128) * nc))) return rc;
    for (int l = 0; l < MAX_LEVELS; ++l) {
        w.f[l] = (c64*)W.mg[2 * l].p;
        w.e[l] = (c64*)W.mg[2 * l + 1].p;
    }
    w.ra = (c128*)W.mg[2 * MAX_LEVELS].p;
    w.rb = (c128*)W.mg[2 * MAX_LEVELS + 1].p;
    w.xw = (c128*)W.mg[2 * MAX_LEVELS + 2].p;
    return launch_vcycle<float>(op, (const c64*)f, nullptr, 0, (c64*)e, nullptr, nrhs, nullptr, 0, w, s);
}

int helm_resample(const float* in, int nz, int nx, float* out, int mz, int mx, void* stream) {
    if (!in || !out || nz < 1 || nx < 1 || mz < 1 || mx < 1) return fail(HELM_EINVAL, "helm_resample: bad arguments");
    const long n = (long)mz * mx;
    hipLaunchKernelGGL(k_resample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, in, nz, nx,
                       out, mz, mx);
    HELM_CHECK_LAUNCH();
    return HELM_OK;
}

int helm_coarse_roots(helm_op_t op, double* roots, int* n) {
    if (!op || !n) return fail(HELM_EINVAL, "helm_coarse_roots: bad arguments");
    if (roots)
        for (size_t i = 0; i < op->roots.size(); ++i) {
            roots[2 * i] = op->roots[i].re;
            roots[2 * i + 1] = op->roots[i].im;
        }
    *n = (int)op->roots.size();
    return HELM_OK;
}

int helm_solve(const helm_op_t* ops, int nops, const int* rhs_op, const void* rhs, void* x, int nrhs, double tol,
               const helm_solve_opts* opt, int* iters, double* relres, int* status, void* stream) {
    if (!ops || nops <= 0 || nrhs < 0) return fail(HELM_EINVAL, "helm_solve: bad arguments");
    if (nrhs == 0) return HELM_OK;   // an empty batch: the buffers may be NULL
    if (!rhs || !x) return fail(HELM_EINVAL, "helm_solve: NULL buffer");
    for (int i = 0; i < nops; ++i)
        if (!ops[i]) return fail(HELM_EINVAL, "helm_solve: ops[%d] is NULL", i);
    if (!(tol > 0)) return fail(HELM_EINVAL, "helm_solve: tol must be positive");
    helm_solve_opts o;
    memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (o.precond < HELM_PRECOND_MG || o.precond > HELM_PRECOND_CNN_VU)
        return fail(HELM_EINVAL, "helm_solve: unknown preconditioner %d", o.precond);
    const bool cnn = o.precond == HELM_PRECOND_CNN || o.precond == HELM_PRECOND_CNN_VU;
    if (cnn && !o.net) return fail(HELM_EINVAL, "helm_solve: CNN preconditioner needs opts.net");
    if (o.restart <= 0) o.restart = cnn ? 10 : 20;
    if (o.restart > MAX_RESTART) return fail(HELM_EINVAL, "helm_solve: restart must be <= %d", MAX_RESTART);
    if (o.maxit <= 0) o.maxit = 300;
    if (o.streams < 0 || o.streams > 2) return fail(HELM_EINVAL, "helm_solve: streams must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_mutex);
    hipStream_t s = (hipStream_t)stream;
    hipStream_t us = s;
    if (o.use_graph) {
        s = graph_stream();
        if (!s) return fail(HELM_EHIP, "helm_solve: could not create the graph stream");
        hipEvent_t ev;
        HELM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HELM_HIP(hipEventRecord(ev, us));
        HELM_HIP(hipStreamWaitEvent(s, ev, 0));
        (void)hipEventDestroy(ev);
    }
    if (o.krylov_dtype == HELM_C128)
        return solve_impl<double>(ops, nops, rhs_op, rhs, x, nrhs, tol, o, iters, relres, status, s);
    if (o.krylov_dtype == HELM_C64)
        return solve_impl<float>(ops, nops, rhs_op, rhs, x, nrhs, tol, o, iters, relres, status, s);
    return fail(HELM_EINVAL, "helm_solve: krylov_dtype %d", o.krylov_dtype);
}

}  // extern "C"
