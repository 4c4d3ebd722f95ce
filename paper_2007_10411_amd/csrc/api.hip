// C ABI of the JFNK library: context set-up, operator entry points, flexible
// restarted GMRES and the inexact Newton step (section 2.5 of the paper,
// equations 5, 8 and 9).  Host orchestration only; every arithmetic step on the
// state runs in the kernels of stencil2d.hip and vec.hip.

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "jfnk_internal.hpp"
#include "reduce.hpp"

namespace jfnk {

namespace {
thread_local std::string g_err;

// device-scalar layout (doubles)
constexpr int M = kMaxDots;
constexpr int O_H = 0;
constexpr int O_HRAW = O_H + (M + 1) * M;
constexpr int O_CS = O_HRAW + (M + 1) * M;
constexpr int O_SN = O_CS + M;
constexpr int O_G = O_SN + M;
constexpr int O_Y = O_G + M + 1;
constexpr int O_H1 = O_Y + M;
constexpr int O_H2 = O_H1 + M;
constexpr int O_R = O_H2 + M;         // one-reduction step: norms r_c of the basis vectors before normalization
constexpr int O_CO = O_R + M;         //   and the update coefficients (a, e, 1/r, c_w)
constexpr int O_S = O_CO + 2 * M + 2; // misc scalars
enum { S_UNORM2 = 0, S_VNORM2, S_EPS, S_WNORM2, S_WNORM, S_RES, S_BETA2, S_BETA, S_TMP, S_SLOT0 = 10, S_COUNT = 18 };
constexpr int kScal = O_S + S_COUNT;

double* ds(jfnk_ctx* c, int off) { return c->dscal + off; }
double* sc(jfnk_ctx* c, int which) { return c->dscal + O_S + which; }

template <typename T> T* Vb(jfnk_ctx* c);
template <> double* Vb<double>(jfnk_ctx* c) { return c->V64; }
template <> float* Vb<float>(jfnk_ctx* c) { return c->V32; }
template <typename T> T* Zb(jfnk_ctx* c);
template <> double* Zb<double>(jfnk_ctx* c) { return c->Z64; }
template <> float* Zb<float>(jfnk_ctx* c) { return c->Z32; }
template <typename T> T* NUb(jfnk_ctx* c);
template <> double* NUb<double>(jfnk_ctx* c) { return c->nu64; }
template <> float* NUb<float>(jfnk_ctx* c) { return c->nu32; }
template <typename T> T* TA(jfnk_ctx* c);
template <> double* TA<double>(jfnk_ctx* c) { return c->t64a; }
template <> float* TA<float>(jfnk_ctx* c) { return c->t32a; }
template <typename T> T* TB(jfnk_ctx* c);
template <> double* TB<double>(jfnk_ctx* c) { return c->t64b; }
template <> float* TB<float>(jfnk_ctx* c) { return c->t32b; }
template <typename T> constexpr int is32() { return sizeof(T) == 4 ? 1 : 0; }
int tv(jfnk_ctx* c, int stage, int f32) { return c->tune[stage * 2 + f32]; }

template <typename T> T* DB(jfnk_ctx* c);
template <> double* DB<double>(jfnk_ctx* c) { return c->d64; }
template <> float* DB<float>(jfnk_ctx* c) { return c->d32; }

// operator dispatch: 2D tiled kernels (tuned tile height) or the 3D two-pass kernels
template <typename T>
hipError_t op_F(jfnk_ctx* c, const T* u, const T* f, T* out, int what) {
    if (c->geo.dim == 3) return launch3_apply_F<T>(c->geo, u, f, out, what, DB<T>(c), c->stream);
    return launch_apply_F<T>(c->geo, u, f, out, what, c->stream, tv(c, 0, is32<T>()));
}
template <typename T>
hipError_t op_jv(jfnk_ctx* c, const T* u, const T* v, double eps, const double* eps_dev, T* out) {
    if (c->geo.dim == 3) {
        if constexpr (std::is_same<T, float>::value) {
            if (c->jv3_single && c->geo.W == 2) return launch3_jv_fused(c->geo, u, v, eps, eps_dev, out, c->stream);
        }
        return launch3_jv<T>(c->geo, u, v, eps, eps_dev, out, DB<T>(c), c->stream);
    }
    return launch_jv<T>(c->geo, u, v, eps, eps_dev, out, c->stream, tv(c, 1, is32<T>()));
}
template <typename T>
hipError_t op_frozen_nu(jfnk_ctx* c, const T* u, T* nu) {
    if (c->geo.dim == 3) return launch3_frozen_nu<T>(c->geo, u, nu, c->stream);
    return launch_frozen_nu<T>(c->geo, u, nu, c->stream);
}
template <typename T>
hipError_t op_pc_diag(jfnk_ctx* c, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea) {
    if (c->geo.dim == 3) return launch3_pc_diag<T>(c->geo, nu, vj, div, z, ea, c->stream);
    return launch_pc_diag<T>(c->geo, nu, vj, div, z, ea, c->stream);
}
template <typename T>
hipError_t op_pc_sweep(jfnk_ctx* c, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                       const EpsArgs& ea) {
    if (c->geo.dim == 3) return launch3_pc_sweep<T>(c->geo, u, nu, r, zin, zout, ea, c->stream);
    return launch_pc_sweep<T>(c->geo, u, nu, r, zin, zout, ea, c->stream, tv(c, 2, is32<T>()));
}

template <typename T> constexpr double eps_mach();
template <> constexpr double eps_mach<double>() { return 2.220446049250313e-16; }   // 2^-52
template <> constexpr double eps_mach<float>() { return 1.1920928955078125e-07; }   // 2^-23

// ---- timing ----
struct TimedLaunch {
    jfnk_ctx* c;
    int cls;
    bool active;
    TimedLaunch(jfnk_ctx* c_, int cls_, double bytes = 0.0)
        : c(c_), cls(cls_), active(c_->timing.on && ((c_->timing.mask >> cls_) & 1u)) {
        if (!active) return;
        c->timing.bytes[cls] += bytes;
        auto& T = c->timing;
        if ((int)T.ev[cls].size() < 2 * (T.used[cls] + 1)) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                active = false;
                return;
            }
            T.ev[cls].push_back(a);
            T.ev[cls].push_back(b);
        }
        (void)hipEventRecord(T.ev[cls][2 * T.used[cls]], c->stream);
    }
    ~TimedLaunch() {
        if (!active) return;
        auto& T = c->timing;
        (void)hipEventRecord(T.ev[cls][2 * T.used[cls] + 1], c->stream);
        T.used[cls]++;
        T.launches[cls]++;
    }
};

// learned preconditioner of the context's dimension
hipError_t net_run(jfnk_ctx* c, const float* r, float* z, bool bf16, const EpsArgs* ea = nullptr,
                   const double* rpart = nullptr, int rnblk = 0) {
    const float hdt = (float)(0.5 * c->prob.dt);
    if (c->net.dim == 3)
        return net3_apply(c->net, c->geo.nx, c->geo.ny, c->geo.nz, c->nf, hdt, r, z, bf16, c->stream, ea, rpart,
                          rnblk);
    return net_apply(c->net, c->geo.nx, c->geo.nz, c->nf, hdt, r, z, bf16, c->stream, ea, rpart, rnblk);
}

void resolve_timing(jfnk_ctx* c) {
    auto& T = c->timing;
    for (int k = 0; k < KC_COUNT; ++k) {
        for (int i = 0; i < T.used[k]; ++i) {
            float ms = 0.f;
            (void)hipEventSynchronize(T.ev[k][2 * i + 1]);
            if (hipEventElapsedTime(&ms, T.ev[k][2 * i], T.ev[k][2 * i + 1]) == hipSuccess) T.ms[k] += ms;
        }
        T.used[k] = 0;
    }
}

// Deterministic non-zero fill of the autotuner's operands (strain, closure and
// mixing-length branches all active): x_i = 0.01 (h(i) / 2^32 - 1/2), h an integer hash.
template <typename T>
__global__ void k_tune_fill(T* x, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned h = (unsigned)i * 2654435761u;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = T(0.01 * ((double)h * (1.0 / 4294967296.0) - 0.5));
}

// ---- background and surface flux set-up (section 2.1, section 3.2) ----
__global__ void k_background(Geo g, jfnk_problem p, double* pbar, double* dpbar, double* sflux, float* pbar32,
                             float* dpbar32, float* sflux32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < g.nz) {
        const double z = (t + 0.5) * g.dz;
        const double thb = p.theta0 + g.beta * z;
        double pb;
        if (g.beta > 0.0)
            pb = p.cp - (p.g / g.beta) * log1p(g.beta * z / p.theta0);
        else
            pb = p.cp - p.g * z / p.theta0;
        const double dpb = -p.g / thb;
        pbar[t] = pb;
        dpbar[t] = dpb;
        pbar32[t] = (float)pb;
        dpbar32[t] = (float)dpb;
    }
    const int nxy = g.nx * g.ny;
    if (sflux && t < nxy) {
        // the cell centre is rounded on its own, as the strip definition reads
        // (no multiply-add fused into the strip test, whose edges can fall
        // exactly on a centre)
#pragma clang fp contract(off)
        const int i = t % g.nx;
        const double x = (i + 0.5) * g.dx;
        double H = 0.0;
        if (p.h0 != 0.0 && p.bc_vertical != JFNK_BC_PERIODIC) {
            const double half = 0.5 * p.strip_width;
            if (p.strip_shape == 0) {
                H = fabs(x - p.strip_center) <= half ? p.h0 : 0.0;
            } else {
                const double xp = (x - p.strip_center) / half;
                H = 0.5 * p.h0 * (tanh((xp + 1.0) / p.strip_xi) - tanh((xp - 1.0) / p.strip_xi));
            }
        }
        const double rho0 = p.p_ref / (p.rgas * p.theta0);
        const double q = H / (rho0 * p.cp) / g.dz;
        sflux[t] = q;
        sflux32[t] = (float)q;
    }
}

template <typename T>
int norm2_to(jfnk_ctx* c, const T* x, long long n, double* out_dev) {
    const int nb = red_blocks(n);
    JFNK_HIP(launch_norm2_partial<T>(x, n, c->partials, nb, c->stream));
    JFNK_HIP(launch_reduce_partials(c->partials, nb, 1, 1, out_dev, 0, c->stream));
    return JFNK_OK;
}

int read_scalars(jfnk_ctx* c, int first, int count) {
    JFNK_HIP(hipMemcpyAsync(c->hscal + first, sc(c, first), count * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    JFNK_HIP(hipStreamSynchronize(c->stream));
    return JFNK_OK;
}

template <typename T>
int apply_pc(jfnk_ctx* c, int pc, const T* u, T* vj, const double* div, T* z, int sweeps, T* scratch,
             const EpsArgs& ea, const double* vpart = nullptr);

// Internal Jv mode of the nonlinear preconditioning: the finite-difference
// Jacobian of R~(u) = P^{-1}(u) R(u), [R~(u + eps v) - R~(u)] / eps, with R~(u)
// cached in nl64 and f(u^n) in f64 (FP64 only).
constexpr int kJvNlpc = 3;

// R~(w) = P^{-1}(w) R(w) into out (rbuf receives R(w), scratch is the
// preconditioner's ping-pong vector); the eddy viscosity is frozen at w.
int rtilde64(jfnk_ctx* c, const double* w, double* rbuf, double* out, double* scratch, int sweeps) {
    {
        TimedLaunch tl(c, KC_RESIDUAL);
        JFNK_HIP(op_F<double>(c, w, c->f64, rbuf, 2));
    }
    JFNK_HIP(op_frozen_nu<double>(c, w, NUb<double>(c)));
    return apply_pc<double>(c, JFNK_PC_PHYSICS, w, rbuf, nullptr, out, sweeps, scratch, EpsArgs());
}

// Jv with eps from the device scalar (stable / literal) or eps = 0 (analytic)
template <typename T>
int apply_jv(jfnk_ctx* c, int mode, const T* u, const T* v, const double* eps_dev, double eps_host, T* out) {
    if (mode == kJvNlpc) {
        if constexpr (std::is_same<T, double>::value) {
            double e = eps_host;
            if (eps_dev) {
                JFNK_HIP(hipMemcpyAsync(&c->hscal[S_TMP], eps_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
                JFNK_HIP(hipStreamSynchronize(c->stream));
                e = c->hscal[S_TMP];
            }
            if (!(e > 0.0)) {
                JFNK_HIP(launch_cast<double, double>(out, v, c->n, 0.0, c->stream));
                return JFNK_OK;
            }
            JFNK_HIP(launch_lincomb<double>(c->t64a, u, v, c->n, 1.0, e, c->stream));
            int rc = rtilde64(c, c->t64a, c->t64b, out, c->nls64, c->nl_sweeps);
            if (rc) return rc;
            JFNK_HIP(launch_lincomb<double>(out, out, c->nl64, c->n, 1.0 / e, -1.0 / e, c->stream));
            return JFNK_OK;
        } else {
            set_error("the nonlinear preconditioning runs in FP64");
            return JFNK_ERR_ARG;
        }
    }
    if (mode == JFNK_JV_LITERAL) {
        double e = eps_host;
        if (eps_dev) {
            JFNK_HIP(hipMemcpyAsync(&c->hscal[S_TMP], eps_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            JFNK_HIP(hipStreamSynchronize(c->stream));
            e = c->hscal[S_TMP];
        }
        if (!(e > 0.0)) {   // v = 0 (the automatic step is 0): J 0 = 0
            JFNK_HIP(launch_cast<T, T>(out, v, c->n, 0.0, c->stream));
            return JFNK_OK;
        }
        T* w1 = TA<T>(c);
        T* w2 = TB<T>(c);
        JFNK_HIP(launch_lincomb<T>(w1, u, v, c->n, 1.0, e, c->stream));
        {
            TimedLaunch tl(c, KC_RESIDUAL);
            JFNK_HIP(op_F<T>(c, w1, nullptr, w2, 2));
        }
        {
            TimedLaunch tl(c, KC_RESIDUAL);
            JFNK_HIP(op_F<T>(c, u, nullptr, w1, 2));
        }
        JFNK_HIP(launch_lincomb<T>(out, w2, w1, c->n, 1.0 / e, -1.0 / e, c->stream));
        return JFNK_OK;
    }
    TimedLaunch tl(c, KC_JV, 3.0 * c->n * sizeof(T));
    if (mode == JFNK_JV_ANALYTIC)
        JFNK_HIP(op_jv<T>(c, u, v, 0.0, nullptr, out));
    else
        JFNK_HIP(op_jv<T>(c, u, v, eps_host, eps_dev, out));
    return JFNK_OK;
}

// eps for direction v at state u: needs ||u||^2 already in S_UNORM2
template <typename T>
int fd_eps_dev(jfnk_ctx* c, const T* v) {
    int rc = norm2_to<T>(c, v, c->n, sc(c, S_VNORM2));
    if (rc) return rc;
    JFNK_HIP(launch_fd_eps(sc(c, S_UNORM2), sc(c, S_VNORM2), std::sqrt(eps_mach<T>()), std::sqrt((double)c->n),
                           sc(c, S_EPS), c->stream));
    return JFNK_OK;
}

EpsArgs eps_args(jfnk_ctx* c, double eps_mach_v) {
    EpsArgs a;
    a.partials = c->epart;
    a.unorm2 = sc(c, S_UNORM2);
    a.vnorm2 = sc(c, S_VNORM2);
    a.eps = sc(c, S_EPS);
    a.sqrt_eps = std::sqrt(eps_mach_v);
    a.sqrt_n = std::sqrt((double)c->n);
    return a;
}

// z = P^{-1} v by the physics preconditioner (nu frozen beforehand) or z = v,
// where v = V_j / *div is first written back into V_j (div may be null).  When
// ea.partials is set, the FD step for direction z is formed on the way.
// vpart (may be null): the per-block partial sums of v^2 that the Arnoldi
// update pass left when it wrote v, from which the learned preconditioner
// takes its input scale.
template <typename T>
int apply_pc(jfnk_ctx* c, int pc, const T* u, T* vj, const double* div, T* z, int sweeps, T* scratch,
             const EpsArgs& ea, const double* vpart) {
    if (pc == JFNK_PC_NONE) {
        TimedLaunch tl(c, KC_PC);
        JFNK_HIP(launch_normalize_copy<T>(vj, c->n, div, z, ea, c->stream));
        return JFNK_OK;
    }
    if (pc == JFNK_PC_LEARNED) {
        if (!std::is_same<T, float>::value || !c->net.ready) {
            set_error("the learned preconditioner needs FP32 vectors and parameters set by jfnk_net_set_params");
            return JFNK_ERR_ARG;
        }
        if (div) JFNK_HIP(launch_scale<T>(vj, c->n, div, c->stream));
        {
            // counted in flops: 2 multiply-adds per weight and point; the last
            // layer leaves the partial sums of ||z||^2 for the FD step
            TimedLaunch tl(c, KC_NET, 2.0 * (c->net.nparam) * c->geo.npts);
            JFNK_HIP(net_run(c, (const float*)vj, (float*)z, true, ea.partials ? &ea : nullptr,
                             div ? nullptr : vpart, cgs_blocks(c->n)));
        }
        return JFNK_OK;
    }
    if (pc != JFNK_PC_PHYSICS) {
        set_error("unsupported preconditioner kind");
        return JFNK_ERR_ARG;
    }
    const T* nu = NUb<T>(c);
    EpsArgs none;
    // ping-pong so that the last sweep lands in z
    T* bufs[2] = {z, scratch};
    int cur = (sweeps % 2 == 0) ? 0 : 1;
    const double npts = (double)c->geo.npts;
    {
        TimedLaunch tl(c, KC_PC, ((div ? 3.0 : 2.0) * c->n + npts) * sizeof(T));
        JFNK_HIP(op_pc_diag<T>(c, nu, vj, div, bufs[cur], sweeps == 0 ? ea : none));
    }
    for (int s = 0; s < sweeps; ++s) {
        TimedLaunch tl(c, KC_PC, (3.0 * c->n + (c->geo.dim + 1) * npts) * sizeof(T));
        JFNK_HIP(op_pc_sweep<T>(c, u, nu, vj, bufs[cur], bufs[1 - cur], s == sweeps - 1 ? ea : none));
        cur = 1 - cur;
    }
    return JFNK_OK;
}

// Judge of a learned-preconditioner solve (c->judge_active < 0 while one runs):
// at the end of a cycle that has not converged, the mean log reduction of the
// residual estimate per iteration so far must reach the physics-based
// preconditioner's (section 2.5.2) on record; a solve that falls short stops
// there (c->judged_out) so that the caller can hand the system to the physics-based
// preconditioner after at most one cycle.
bool judged_short(jfnk_ctx* c, double res_est, double bnorm, int total) {
    if (!(c->judge_active < 0.0) || total < 1 || !(bnorm > 0.0)) return false;
    const double rate = res_est > 0.0 ? std::log(res_est / bnorm) / total : -INFINITY;
    if (rate <= c->judge_active) return false;
    c->judged_out = true;
    return true;
}

// Start of both GMRES forms: frozen coefficients, ||u||^2, x = 0, V_0 = rhs and
// beta = ||rhs|| (g = beta e_1, beta also on the host).  bnorm = 0: nothing
// to solve (info says converged).
template <typename T>
int gmres_begin(jfnk_ctx* c, const T* u, const T* b, T* x, const jfnk_gmres_opts& o, jfnk_gmres_info* info,
                double& bnorm) {
    const long long n = c->n;
    T* V = Vb<T>(c);
    hipStream_t s = c->stream;
    int rc;
    if (o.pc == JFNK_PC_PHYSICS) JFNK_HIP(op_frozen_nu<T>(c, u, NUb<T>(c)));
    if ((rc = norm2_to<T>(c, u, n, sc(c, S_UNORM2)))) return rc;
    JFNK_HIP(hipMemsetAsync(x, 0, n * sizeof(T), s));
    JFNK_HIP(hipMemcpyAsync(V, b, n * sizeof(T), hipMemcpyDeviceToDevice, s));
    if ((rc = norm2_to<T>(c, V, n, sc(c, S_BETA2)))) return rc;
    JFNK_HIP(launch_set_start(sc(c, S_BETA2), ds(c, O_G), sc(c, S_BETA), o.m, s));
    if ((rc = read_scalars(c, S_BETA, 1))) return rc;
    bnorm = c->hscal[S_BETA];
    if (info) {
        info->res0 = bnorm;
        info->res_est = bnorm;
        info->iters = 0;
        info->restarts = 0;
        info->converged = bnorm == 0.0 ? 1 : 0;
    }
    if (!std::isfinite(bnorm)) {
        set_error("non-finite right-hand side norm");
        return JFNK_ERR_NONFINITE;
    }
    return JFNK_OK;
}

// Restart: the true residual r = rhs - J x into V_0, beta = ||r||, g = beta e_1;
// zero when r = 0.
template <typename T>
int gmres_restart(jfnk_ctx* c, const T* u, const T* b, const T* x, const jfnk_gmres_opts& o, bool& zero) {
    const long long n = c->n;
    T* V = Vb<T>(c);
    hipStream_t s = c->stream;
    int rc;
    if (o.jv != JFNK_JV_ANALYTIC && (rc = fd_eps_dev<T>(c, x))) return rc;
    if ((rc = apply_jv<T>(c, o.jv, u, x, sc(c, S_EPS), 0.0, V))) return rc;
    JFNK_HIP(launch_lincomb<T>(V, b, V, n, 1.0, -1.0, s));
    if ((rc = norm2_to<T>(c, V, n, sc(c, S_BETA2)))) return rc;
    JFNK_HIP(launch_set_start(sc(c, S_BETA2), ds(c, O_G), sc(c, S_BETA), o.m, s));
    if ((rc = read_scalars(c, S_BETA, 1))) return rc;
    zero = c->hscal[S_BETA] == 0.0;
    return JFNK_OK;
}

// End of both GMRES forms: the result fields (and the raw Hessenberg matrix of
// the last cycle when asked for), after the stream has drained.
int gmres_end(jfnk_ctx* c, jfnk_gmres_info* info, int m, int total, int restarts, bool converged, double res_est) {
    if (info) {
        info->iters = total;
        info->restarts = restarts;
        info->converged = converged ? 1 : 0;
        info->res_est = res_est;
        if (info->h_out) {
            JFNK_HIP(hipMemcpyAsync(info->h_out, ds(c, O_HRAW), (size_t)(m + 1) * m * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
        }
    }
    JFNK_HIP(hipStreamSynchronize(c->stream));
    return converged ? JFNK_OK : JFNK_NOT_CONVERGED;
}

template <typename T>
int gmres_one_reduction(jfnk_ctx* c, const T* u, const T* b, T* x, const jfnk_gmres_opts& o,
                        jfnk_gmres_info* info);

template <typename T>
int gmres_impl(jfnk_ctx* c, const T* u, const T* b, T* x, const jfnk_gmres_opts& o, jfnk_gmres_info* info) {
    if (o.ortho == JFNK_ORTHO_ONE_REDUCTION && o.m < kDgMaxRows && c->n < (1LL << 30))
        return gmres_one_reduction<T>(c, u, b, x, o, info);
    const long long n = c->n;
    const int m = o.m;
    const int max_iters = o.max_iters > 0 ? o.max_iters : m * o.max_restarts;
    T* V = Vb<T>(c);
    T* Z = Zb<T>(c);
    hipStream_t s = c->stream;
    int rc;
    double bnorm = 0.0;
    if ((rc = gmres_begin<T>(c, u, b, x, o, info, bnorm))) return rc;
    if (bnorm == 0.0) return JFNK_OK;
    const EpsArgs ea = o.jv == JFNK_JV_ANALYTIC ? EpsArgs() : eps_args(c, eps_mach<T>());
    GivensArgs ga;
    ga.H = ds(c, O_H);
    ga.Hraw = ds(c, O_HRAW);
    ga.cs = ds(c, O_CS);
    ga.sn = ds(c, O_SN);
    ga.g = ds(c, O_G);
    ga.h1 = ds(c, O_H1);
    ga.h2 = ds(c, O_H2);
    ga.wnorm = sc(c, S_WNORM);
    ga.res_est = sc(c, S_RES);
    ga.m = m;
    GivensArgs gnone;
    int total = 0, restarts = 0, enqueued = 0;
    bool converged = false;
    double res_est = bnorm;
    // Iteration j+1 is enqueued before the host tests iteration j (two pinned
    // result slots); when j has converged the speculative j+1 is discarded: it
    // only wrote column j+1 of H, g[j+1] and V_{j+2}, Z_{j+1}, none of which the
    // back substitution over the first j+1 columns reads.
    auto enqueue_iter = [&](int j) -> int {
        T* Vj = V + (long long)j * n;
        T* Vn = V + (long long)(j + 1) * n;
        T* Zj = Z + (long long)j * n;
        // v_j = w_j / ||w_j|| (beta at the start of a cycle), z_j = M^-1 v_j, FD step for z_j
        const double* div = j == 0 ? sc(c, S_BETA) : sc(c, S_WNORM);
        int r;
        if ((r = apply_pc<T>(c, o.pc, u, Vj, div, Zj, o.sweeps, Vn, ea))) return r;
        if ((r = apply_jv<T>(c, o.jv, u, Zj, sc(c, S_EPS), 0.0, Vn))) return r;
        if (std::is_same<T, float>::value && c->rec_count && *c->rec_count < c->rec_cap) {
            const long long off = (long long)(*c->rec_count) * n;
            JFNK_HIP(hipMemcpyAsync(c->rec_r + off, Vn, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            JFNK_HIP(hipMemcpyAsync(c->rec_du + off, Zj, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            ++*c->rec_count;
        }
        {
            // classical Gram-Schmidt, twice; the Givens step of column j rides on the last pass
            // dot pass reads V_0..V_j and w; each update pass also writes w
            TimedLaunch tl(c, KC_ARNOLDI, (3.0 * (j + 1) + 5.0) * n * sizeof(T));
            ga.j = j;
            ga.host = c->hscal + S_SLOT0 + 2 * (j & 1);   // (||w||, |g_{j+1}|) for the host's test
            JFNK_HIP(launch_cgs<T>(V, n, j + 1, nullptr, Vn, c->partials, ds(c, O_H1), CGS_DOT, gnone, s));
            JFNK_HIP(launch_cgs<T>(V, n, j + 1, ds(c, O_H1), Vn, c->partials, ds(c, O_H2), CGS_UPD_DOT, gnone, s));
            JFNK_HIP(launch_cgs<T>(V, n, j + 1, ds(c, O_H2), Vn, c->partials, sc(c, S_WNORM2), CGS_UPD_NORM, ga,
                                   s));
        }
        JFNK_HIP(hipEventRecord(c->slot_ev[j & 1], s));
        ++enqueued;
        return JFNK_OK;
    };
    // wait for iteration j and decide whether the cycle stops after it
    auto finish_iter = [&](int j, bool& stop) -> int {
        const int slot = j & 1;
        JFNK_HIP(hipEventSynchronize(c->slot_ev[slot]));
        const double wn = c->hscal[S_SLOT0 + 2 * slot];
        res_est = c->hscal[S_SLOT0 + 2 * slot + 1];
        if (!std::isfinite(wn) || !std::isfinite(res_est)) {
            set_error("non-finite Krylov norm");
            return JFNK_ERR_NONFINITE;
        }
        ++total;
        stop = res_est <= o.tol * bnorm || wn == 0.0 || total >= max_iters;
        return JFNK_OK;
    };
    while (true) {
        int k = 0;
        bool done = false;
        if ((rc = enqueue_iter(0))) return rc;
        for (int j = 0; j < m; ++j) {
            if (j + 1 < m && enqueued < max_iters)
                if ((rc = enqueue_iter(j + 1))) return rc;
            bool stop = false;
            if ((rc = finish_iter(j, stop))) return rc;
            k = j + 1;
            if (stop) {
                done = true;
                break;
            }
        }
        JFNK_HIP(launch_backsolve(ds(c, O_H), ds(c, O_G), k, m, ds(c, O_Y), s));
        JFNK_HIP(launch_axpy_basis<T>(x, Z, n, k, ds(c, O_Y), s));
        if (done) {
            converged = res_est <= o.tol * bnorm;
            break;
        }
        if (judged_short(c, res_est, bnorm, total)) break;
        ++restarts;
        // true residual r = b - J x
        bool zero = false;
        if ((rc = gmres_restart<T>(c, u, b, x, o, zero))) return rc;
        if (zero) {
            converged = true;
            break;
        }
    }
    return gmres_end(c, info, m, total, restarts, converged, res_est);
}

// FGMRES(m) with the one-reduction Arnoldi step (three launches per iteration:
// the reduction pass, its finishing block and the update pass).  Column c of
// the Hessenberg matrix is final one iteration later (iteration c + 1 or, for
// the last column of a cycle, a closing reduction over basis vector c + 1
// alone).  Iterations run up to two ahead of the host's test; a speculative
// iteration only writes columns, rotations and basis vectors past the ones the
// back substitution reads.
template <typename T>
int gmres_one_reduction(jfnk_ctx* c, const T* u, const T* b, T* x, const jfnk_gmres_opts& o,
                        jfnk_gmres_info* info) {
    const long long n = c->n;
    const int m = o.m;
    const int max_iters = o.max_iters > 0 ? o.max_iters : m * o.max_restarts;
    T* V = Vb<T>(c);
    T* Z = Zb<T>(c);
    hipStream_t s = c->stream;
    int rc;
    double bnorm = 0.0;
    if ((rc = gmres_begin<T>(c, u, b, x, o, info, bnorm))) return rc;
    if (bnorm == 0.0) return JFNK_OK;
    const EpsArgs ea = o.jv == JFNK_JV_ANALYTIC ? EpsArgs() : eps_args(c, eps_mach<T>());
    DgArgs da;
    da.H = ds(c, O_H);
    da.Hraw = ds(c, O_HRAW);
    da.cs = ds(c, O_CS);
    da.sn = ds(c, O_SN);
    da.g = ds(c, O_G);
    da.h1 = ds(c, O_H1);
    da.rs = ds(c, O_R);
    da.coef = ds(c, O_CO);
    da.m = m;
    int total = 0, restarts = 0;
    bool converged = false;
    double res_est = bnorm;
    auto slot_of = [](int op) { return op & 3; };
    // the learned preconditioner takes the scale of q~_j from the partial sums
    // of its squares that the update pass of iteration j - 1 leaves
    const bool learned = o.pc == JFNK_PC_LEARNED && std::is_same<T, float>::value;
    // iteration j: z_j = M q~_j, w = A z_j, the reduction (closes column j-1), the update
    auto enqueue_iter = [&](int j) -> int {
        T* Vj = V + (long long)j * n;
        T* Vn = V + (long long)(j + 1) * n;
        T* Zj = Z + (long long)j * n;
        int r;
        if ((r = apply_pc<T>(c, o.pc, u, Vj, nullptr, Zj, o.sweeps, Vn, ea, learned && j > 0 ? c->qpart : nullptr)))
            return r;
        if ((r = apply_jv<T>(c, o.jv, u, Zj, sc(c, S_EPS), 0.0, Vn))) return r;
        if (std::is_same<T, float>::value && c->rec_count && *c->rec_count < c->rec_cap) {
            const long long off = (long long)(*c->rec_count) * n;
            JFNK_HIP(hipMemcpyAsync(c->rec_r + off, Vn, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            JFNK_HIP(hipMemcpyAsync(c->rec_du + off, Zj, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            ++*c->rec_count;
        }
        {
            // the reduction pass reads V_0..V_{j+1}; the update pass reads them and writes two rows
            TimedLaunch tl(c, KC_ARNOLDI, (2.0 * j + 6.0) * n * sizeof(T));
            da.host = c->hscal + S_SLOT0 + 2 * slot_of(j);
            JFNK_HIP(launch_dg_reduce<T>(V, n, j, true, c->partials, da, s));
            JFNK_HIP(hipEventRecord(c->slot_ev[slot_of(j)], s));
            JFNK_HIP(launch_dg_update<T>(V, n, j, da.coef, s, learned ? c->qpart : nullptr));
        }
        return JFNK_OK;
    };
    // closing reduction over q~_k alone: column k-1 becomes final
    auto enqueue_close = [&](int k) -> int {
        TimedLaunch tl(c, KC_ARNOLDI, (k + 1.0) * n * sizeof(T));
        da.host = c->hscal + S_SLOT0 + 2 * slot_of(k);
        JFNK_HIP(launch_dg_reduce<T>(V, n, k, false, c->partials, da, s));
        JFNK_HIP(hipEventRecord(c->slot_ev[slot_of(k)], s));
        return JFNK_OK;
    };
    auto enqueue_op = [&](int op, int kmax) -> int { return op < kmax ? enqueue_iter(op) : enqueue_close(op); };
    while (true) {
        const int kmax = std::min(m, max_iters - total);    // columns of this cycle
        int k = 0;
        bool done = false;
        if ((rc = enqueue_op(0, kmax))) return rc;
        if ((rc = enqueue_op(1, kmax))) return rc;
        for (int col = 0; col < kmax; ++col) {
            if (col + 2 <= kmax && (rc = enqueue_op(col + 2, kmax))) return rc;
            // column col is closed by op col + 1
            const int slot = slot_of(col + 1);
            JFNK_HIP(hipEventSynchronize(c->slot_ev[slot]));
            const double rnext = c->hscal[S_SLOT0 + 2 * slot];
            res_est = c->hscal[S_SLOT0 + 2 * slot + 1];
            if (!std::isfinite(rnext) || !std::isfinite(res_est)) {
                set_error("non-finite Krylov norm");
                return JFNK_ERR_NONFINITE;
            }
            ++total;
            k = col + 1;
            if (res_est <= o.tol * bnorm || rnext == 0.0 || total >= max_iters) {
                done = true;
                break;
            }
        }
        JFNK_HIP(launch_backsolve(ds(c, O_H), ds(c, O_G), k, m, ds(c, O_Y), s));
        JFNK_HIP(launch_axpy_basis<T>(x, Z, n, k, ds(c, O_Y), s));
        if (done) {
            converged = res_est <= o.tol * bnorm;
            break;
        }
        if (judged_short(c, res_est, bnorm, total)) break;
        ++restarts;
        // true residual r = b - J x, the next cycle's (unnormalized) start vector
        bool zero = false;
        if ((rc = gmres_restart<T>(c, u, b, x, o, zero))) return rc;
        if (zero) {
            converged = true;
            break;
        }
    }
    return gmres_end(c, info, m, total, restarts, converged, res_est);
}

// Krylov solve of J(u) x = b with the preconditioner of go.pc.  The learned
// preconditioner is judged by the physics-based one (section 2.5.2): it runs
// only when a physics-preconditioned solve of this context is on record, and
// stops at the end of the first cycle whose mean log residual reduction per
// iteration falls short of that solve's; the system is then solved again with
// the physics-based preconditioner, as it is when no record exists or the
// learned solve does not converge or breaks down (gi->fallback = 1, the learned
// attempt's iterations added to *spent).  Once a judged learned solve has
// fallen back, *benched (when given) keeps the remaining solves of the caller's
// step on the physics-based preconditioner.  go.no_judge = 1 runs the learned
// solve unjudged, falling back only when it does not converge; 2 returns the
// learned solve's outcome as it is (no fallback).  Every
// physics-preconditioned solve that converges updates the record.
template <typename T>
int krylov_solve(jfnk_ctx* c, const T* u, const T* b, T* x, jfnk_gmres_opts go, jfnk_gmres_info* gi, int* spent,
                 bool* benched = nullptr) {
    gi->fallback = 0;
    gi->res_true = -1.0;
    if (go.pc == JFNK_PC_LEARNED) {
        if (go.no_judge || (c->judge_rate < 0.0 && !(benched && *benched))) {
            c->judge_active = go.no_judge ? 0.0 : c->judge_rate;
            c->judged_out = false;
            int rc = gmres_impl<T>(c, u, b, x, go, gi);
            c->judge_active = 0.0;
            if (go.no_judge == 2) return rc;   // the learned solve's own outcome, no fallback
            if (rc < 0 && rc != JFNK_ERR_NONFINITE) return rc;   // a non-finite learned solve falls back
            if (rc == JFNK_OK && !c->judged_out) {
                // a nonlinear preconditioner can break the Arnoldi process down
                // (a direction with a vanishing image): accept only a finite x
                double x2 = 0.0;
                if ((rc = norm2_to<T>(c, x, c->n, sc(c, S_TMP)))) return rc;
                if ((rc = read_scalars(c, S_TMP, 1))) return rc;
                x2 = c->hscal[S_TMP];
                if (std::isfinite(x2)) return JFNK_OK;
            }
            if (spent) *spent += gi->iters;
            if (benched && !go.no_judge) *benched = true;
        }
        gi->fallback = 1;
        go.pc = JFNK_PC_PHYSICS;
    }
    const int fb = gi->fallback;
    const int rc = gmres_impl<T>(c, u, b, x, go, gi);
    gi->fallback = fb;
    if (rc == JFNK_OK && go.pc == JFNK_PC_PHYSICS && gi->iters > 0 && gi->res0 > 0.0 && gi->res_est > 0.0)
        c->judge_rate = std::log(gi->res_est / gi->res0) / gi->iters;
    return rc;
}

// Autotuner: every compiled tile height (4, 8, 16 rows of 64 points) of the
// three stencil stages, and the row-marching residual and Jv over chunks of 32,
// 64 and 256 rows, in both precisions, are timed with HIP events on this
// context's grid (one warm-up launch, then the fastest of three groups of five
// timed launches, on the workspace vectors filled first with a deterministic
// non-zero pattern); the fastest candidate is kept for the context, the
// default 64 x 8 tile or else the lowest variant when within 3% of it.
template <typename T>
int tune_precision(jfnk_ctx* c, hipEvent_t e0, hipEvent_t e1) {
    T* V = Vb<T>(c);
    T* Z = Zb<T>(c);
    const long long n = c->n;
    hipStream_t s = c->stream;
    hipLaunchKernelGGL((k_tune_fill<T>), dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, s, V, 2 * n);
    JFNK_HIP(hipGetLastError());
    JFNK_HIP(launch_frozen_nu<T>(c->geo, V, NUb<T>(c), s));
    EpsArgs none;
    for (int stage = 0; stage < 3; ++stage) {
        float tvar[6];
        // tiles 64 x 4/8/16 (variants 0-2); row marching over 32/64/256 rows (3-5) for F and Jv
        const int nvar = stage < 2 ? 6 : 3;
        for (int var = 0; var < nvar; ++var) {
            tvar[var] = 1e30f;
            if (stage == 1 && sizeof(T) == 8 && var == 2) continue;   // exceeds the LDS of a CU
            auto launch = [&]() -> hipError_t {
                if (stage == 0) return launch_apply_F<T>(c->geo, V, nullptr, Z, 0, s, var);
                if (stage == 1) return launch_jv<T>(c->geo, V, V + n, 1e-6, nullptr, Z, s, var);
                return launch_pc_sweep<T>(c->geo, V, NUb<T>(c), V + n, V, Z, none, s, var);
            };
            JFNK_HIP(launch());
            float ms = 1e30f;             // fastest of three groups of five launches
            for (int rep = 0; rep < 3; ++rep) {
                JFNK_HIP(hipEventRecord(e0, s));
                for (int k = 0; k < 5; ++k) JFNK_HIP(launch());
                JFNK_HIP(hipEventRecord(e1, s));
                JFNK_HIP(hipEventSynchronize(e1));
                float t = 0.f;
                JFNK_HIP(hipEventElapsedTime(&t, e0, e1));
                ms = t < ms ? t : ms;
            }
            tvar[var] = ms;
        }
        // near-ties (within 3%) go to the default 64 x 8 tile, then to the lowest
        // variant, so that timing noise does not flip the choice between runs
        float best = 1e30f;
        for (int var = 0; var < nvar; ++var) best = tvar[var] < best ? tvar[var] : best;
        int bestv = 1;
        if (tvar[1] > 1.03f * best)
            for (int var = 0; var < nvar; ++var)
                if (tvar[var] <= 1.03f * best) {
                    bestv = var;
                    break;
                }
        c->tune[stage * 2 + is32<T>()] = bestv;
    }
    return JFNK_OK;
}

bool valid_problem(const jfnk_problem* p, std::string& why) {
    if (!p) return why = "null problem", false;
    if (p->dim != 2 && p->dim != 3) return why = "dim must be 2 or 3", false;
    if (p->nx < 8 || p->nz < 8 || (p->dim == 2 && p->ny != 1) || (p->dim == 3 && p->ny < 8))
        return why = "grid below 8 points in a direction (or ny != 1 in 2D)", false;
    if (p->dim == 3 && !(p->ly > 0)) return why = "non-positive domain size", false;
    if (!(p->dt > 0) || !(p->lx > 0) || !(p->lz > 0)) return why = "non-positive dt or domain size", false;
    if (p->dd_p != 2 && p->dd_p != 3) return why = "dd_p must be 2 or 3", false;
    if (p->bc_lateral != JFNK_BC_FREE_SLIP && p->bc_lateral != JFNK_BC_PERIODIC)
        return why = "bc_lateral must be free-slip or periodic", false;
    if (p->bc_vertical < 0 || p->bc_vertical > 2) return why = "invalid bc_vertical", false;
    if (p->closure < 0 || p->closure > 3) return why = "invalid closure", false;
    if (p->closure == JFNK_CLOSURE_DEARDORFF && (!(p->cs >= 0) || !(p->n_bv >= 0)))
        return why = "the anisotropic closure needs cs >= 0 and n_bv >= 0", false;
    if (p->closure == JFNK_CLOSURE_SMAGORINSKY && !(p->pr_t > 0)) return why = "pr_t must be positive", false;
    return true;
}

}  // namespace

// Device geometry and coefficients of a problem (grid, boundary kinds, physical
// constants, closure constants).
void fill_geo(const jfnk_problem& p, Geo& g) {
    g.dim = p.dim;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.npts = (long long)p.nx * p.ny * p.nz;
    g.bcl = p.bc_lateral;
    g.bcv = p.bc_vertical;
    g.W = p.dd_p == 3 ? 4 : 2;
    g.dx = p.lx / p.nx;
    g.dy = p.ly / p.ny;
    g.dz = p.lz / p.nz;
    g.idx = 1.0 / g.dx;
    g.idy = 1.0 / g.dy;
    g.idz = 1.0 / g.dz;
    g.two_dt = 2.0 / p.dt;
    g.theta0 = p.theta0;
    g.g_theta0 = p.g / p.theta0;
    g.kappa = p.kappa_div > 0 ? p.kappa_div : p.rgas / p.cv;
    g.kappa_cp = g.kappa * p.cp;
    g.beta = p.n_bv * p.n_bv * p.theta0 / p.g;
    g.closure = p.closure;
    const double delta = p.dim == 2 ? std::sqrt(g.dx * g.dz) : std::cbrt(g.dx * g.dy * g.dz);
    g.smag = (p.cs * delta) * (p.cs * delta);
    g.inv_pr = p.pr_t > 0 ? 1.0 / p.pr_t : 0.0;
    g.dd_ah = g.dd_av = g.dd_ch = g.dd_cv = g.dd_b = g.dd_delta = g.dd_inv_nu = 0.0;
    if (p.closure == JFNK_CLOSURE_DEARDORFF) {
        // eps^(1/3) = (cs Delta)^(2/3) 2^(1/6) |S|, so every coefficient is linear in |S|
        // below the mixing-length cap; the horizontal scale sqrt(dx dy) (dy = dx in 2D)
        const double gm = std::cbrt((p.cs * delta) * (p.cs * delta)) * std::pow(2.0, 1.0 / 6.0);
        const double c43 = std::pow(p.cs, 4.0 / 3.0);
        const double dh = p.dim == 3 ? std::sqrt(g.dx * g.dy) : g.dx;
        g.dd_ah = c43 * gm * std::pow(dh, 4.0 / 3.0);
        g.dd_av = c43 * gm * std::pow(g.dz, 4.0 / 3.0);
        g.dd_ch = 2.0 * g.dd_ah / dh;
        g.dd_cv = 2.0 * g.dd_av / g.dz;
        g.dd_delta = delta;
        g.dd_b = p.n_bv > 0 ? 0.75 * std::pow(2.0, 2.0 / 3.0) * std::cbrt((p.cs * delta) * (p.cs * delta)) *
                                   std::cbrt(delta) / p.n_bv
                             : 0.0;
        g.dd_inv_nu = g.smag > 0 ? 1.0 / (g.smag * std::sqrt(2.0)) : 0.0;
    }
    g.k_m = p.k_m;
    g.k_h = p.k_h;
    g.convection = p.convection;
    g.energy_test = p.energy_test;
    GeoF& f = g.f;
    f.idx = (float)g.idx;
    f.idy = (float)g.idy;
    f.idz = (float)g.idz;
    f.two_dt = (float)g.two_dt;
    f.theta0 = (float)g.theta0;
    f.g_theta0 = (float)g.g_theta0;
    f.kappa = (float)g.kappa;
    f.kappa_cp = (float)g.kappa_cp;
    f.beta = (float)g.beta;
    f.smag_s2 = (float)g.smag * 1.4142135623730951f;
    f.inv_pr = (float)g.inv_pr;
    f.dd_ah = (float)g.dd_ah;
    f.dd_av = (float)g.dd_av;
    f.dd_ch = (float)g.dd_ch;
    f.dd_cv = (float)g.dd_cv;
    f.dd_b = (float)g.dd_b;
    f.dd_delta = (float)g.dd_delta;
}

void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    return JFNK_ERR_HIP;
}

}  // namespace jfnk

using namespace jfnk;

extern "C" {

const char* jfnk_last_error(void) { return g_err.c_str(); }

int jfnk_create(const jfnk_problem* p, int32_t max_m, void* stream, jfnk_ctx** out) {
    std::string why;
    if (!out) {
        set_error("null output pointer");
        return JFNK_ERR_ARG;
    }
    *out = nullptr;
    if (!valid_problem(p, why)) {
        set_error(why);
        return JFNK_ERR_ARG;
    }
    if (max_m < 1 || max_m + 1 > kMaxDots) {
        set_error("max_m must be in [1, 63]");
        return JFNK_ERR_ARG;
    }
    jfnk_ctx* c = new jfnk_ctx();
    c->prob = *p;
    c->stream = (hipStream_t)stream;
    c->max_m = max_m;
    JFNK_HIP(hipGetDevice(&c->device));
    fill_geo(*p, c->geo);
    Geo& g = c->geo;
    c->nf = p->dim == 2 ? 4 : 5;
    c->n = c->nf * g.npts;
    const long long n = c->n;
    const size_t nb64 = n * sizeof(double), nb32 = n * sizeof(float);
    auto fail = [&](hipError_t e, const char* what) {
        jfnk_destroy(c);
        return hip_fail(e, what);
    };
#define ALLOC(ptr, bytes)                                         \
    do {                                                          \
        hipError_t e_ = hipMalloc((void**)&(ptr), (bytes));       \
        if (e_ != hipSuccess) return fail(e_, "hipMalloc " #ptr); \
    } while (0)
    ALLOC(c->V64, (size_t)(max_m + 1) * nb64);
    ALLOC(c->Z64, (size_t)max_m * nb64);
    ALLOC(c->V32, (size_t)(max_m + 1) * nb32);
    ALLOC(c->Z32, (size_t)max_m * nb32);
    ALLOC(c->f64, nb64);
    ALLOC(c->R64, nb64);
    ALLOC(c->nl64, nb64);
    ALLOC(c->nls64, nb64);
    ALLOC(c->t64a, nb64);
    ALLOC(c->t64b, nb64);
    ALLOC(c->b64, nb64);
    ALLOC(c->x64, nb64);
    const size_t next = (size_t)(g.nx + 2 * g.W) * (g.nz + 2 * g.W) * (g.dim == 3 ? (g.ny + 2 * g.W) : 1);
    ALLOC(c->nu64, next * sizeof(double));
    ALLOC(c->u32, nb32);
    ALLOC(c->b32, nb32);
    ALLOC(c->x32, nb32);
    ALLOC(c->t32a, nb32);
    ALLOC(c->t32b, nb32);
    ALLOC(c->nu32, next * sizeof(float));
    if (g.dim == 3) {
        ALLOC(c->d64, 9 * next * sizeof(double));
        ALLOC(c->d32, 9 * next * sizeof(float));
    }
    const size_t nbg = (size_t)2 * g.nz + (size_t)g.nx * g.ny;
    ALLOC(c->bg64, nbg * sizeof(double));
    ALLOC(c->bg32, nbg * sizeof(float));
    ALLOC(c->partials, (size_t)kMaxPartials * kMaxDots * sizeof(double));
    ALLOC(c->dscal, kScal * sizeof(double));
    {
        const long long tiles = (long long)((g.nx + 63) / 64) * ((g.nz + 7) / 8) * (g.dim == 3 ? g.ny : 1);
        // the network's last layer: one partial per 64 x 4 tile (per plane in 3D)
        const long long conv = (long long)((g.nx + 63) / 64) *
                               (g.dim == 3 ? (long long)((g.ny + 3) / 4) * g.nz : (long long)((g.nz + 3) / 4));
        const long long ne = std::max(std::max(tiles, conv), (g.npts + 255) / 256) + 1024;
        ALLOC(c->epart, (size_t)ne * sizeof(double));
        ALLOC(c->qpart, (size_t)1024 * sizeof(double));   // one per block of the update pass (at most 1024)
    }
#undef ALLOC
    {
        // fine-grained (coherent) so that kernels can write the convergence
        // scalars straight to the host
        hipError_t e = hipHostMalloc((void**)&c->hscal, S_COUNT * sizeof(double), hipHostMallocCoherent);
        if (e != hipSuccess) return fail(e, "hipHostMalloc");
        for (int k = 0; k < 4; ++k) {
            e = hipEventCreateWithFlags(&c->slot_ev[k], hipEventDisableTiming);
            if (e != hipSuccess) return fail(e, "hipEventCreate");
        }
    }
    g.pbar64 = c->bg64;
    g.dpbar64 = c->bg64 + g.nz;
    g.sflux64 = c->bg64 + 2 * g.nz;
    g.pbar32 = c->bg32;
    g.dpbar32 = c->bg32 + g.nz;
    g.sflux32 = c->bg32 + 2 * g.nz;
    {
        hipError_t e = hipMemsetAsync(c->dscal, 0, kScal * sizeof(double), c->stream);
        if (e != hipSuccess) return fail(e, "hipMemsetAsync");
        const int cnt = std::max(g.nz, g.nx * g.ny);
        hipLaunchKernelGGL(k_background, dim3((cnt + 255) / 256), dim3(256), 0, c->stream, g, *p,
                           (double*)g.pbar64, (double*)g.dpbar64, (double*)g.sflux64, (float*)g.pbar32,
                           (float*)g.dpbar32, (float*)g.sflux32);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(e, "k_background");
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(e, "hipStreamSynchronize");
    }
    *out = c;
    return JFNK_OK;
}

int jfnk_destroy(jfnk_ctx* c) {
    if (!c) return JFNK_OK;
    (void)hipStreamSynchronize(c->stream);
    void* ptrs[] = {c->V64, c->Z64, c->V32, c->Z32, c->f64, c->R64, c->nl64, c->nls64, c->t64a, c->t64b, c->b64, c->x64, c->nu64, c->d64, c->d32, c->u32, c->b32,
                    c->x32, c->t32a, c->t32b, c->nu32, c->bg64, c->bg32, c->partials, c->dscal, c->epart, c->qpart};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    {
        NetBuffers& nb = c->net;
        void* np_[] = {nb.theta, nb.grad, nb.m, nb.v, nb.wt, nb.wbf, nb.s, nb.partials, nb.scal, nb.loss,
                       nb.act, nb.pre, nb.a0, nb.z, nb.g0, nb.g1, nb.wpart, nb.abf};
        for (void* q : np_)
            if (q) (void)hipFree(q);
    }
    if (c->hscal) (void)hipHostFree(c->hscal);
    for (int k = 0; k < 4; ++k)
        if (c->slot_ev[k]) (void)hipEventDestroy(c->slot_ev[k]);
    for (int k = 0; k < KC_COUNT; ++k)
        for (auto e : c->timing.ev[k]) (void)hipEventDestroy(e);
    delete c;
    return JFNK_OK;
}

int jfnk_set_stream(jfnk_ctx* c, void* stream) {
    if (!c) {
        set_error("null context");
        return JFNK_ERR_ARG;
    }
    c->stream = (hipStream_t)stream;
    return JFNK_OK;
}

int jfnk_apply_F(jfnk_ctx* c, jfnk_dtype dt, int32_t what, const void* u, const void* f, void* out) {
    if (!c || !u || !out || what < 0 || what > 2) {
        set_error("invalid argument to jfnk_apply_F");
        return JFNK_ERR_ARG;
    }
    TimedLaunch tl(c, KC_RESIDUAL);
    if (dt == JFNK_F64)
        JFNK_HIP(op_F<double>(c, (const double*)u, (const double*)f, (double*)out, what));
    else if (dt == JFNK_F32)
        JFNK_HIP(op_F<float>(c, (const float*)u, (const float*)f, (float*)out, what));
    else {
        set_error("invalid dtype");
        return JFNK_ERR_ARG;
    }
    return JFNK_OK;
}

int jfnk_rhs(jfnk_ctx* c, const double* u_n, double* f) { return jfnk_apply_F(c, JFNK_F64, 1, u_n, nullptr, f); }

int jfnk_residual(jfnk_ctx* c, const double* u, const double* f, double* R) {
    return jfnk_apply_F(c, JFNK_F64, 2, u, f, R);
}

int jfnk_jv(jfnk_ctx* c, jfnk_dtype dt, jfnk_jv_mode mode, const void* u, const void* v, double eps, void* Jv) {
    if (!c || !u || !v || !Jv || mode < 0 || mode > 2) {
        set_error("invalid argument to jfnk_jv");
        return JFNK_ERR_ARG;
    }
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        const double* edev = nullptr;
        if (mode != JFNK_JV_ANALYTIC && !(eps > 0)) {
            int rc = norm2_to<T>(c, (const T*)u, c->n, sc(c, S_UNORM2));
            if (rc) return rc;
            if ((rc = fd_eps_dev<T>(c, (const T*)v))) return rc;
            edev = sc(c, S_EPS);
        }
        return apply_jv<T>(c, mode, (const T*)u, (const T*)v, edev, eps, (T*)Jv);
    };
    if (dt == JFNK_F64) return run(double(0));
    if (dt == JFNK_F32) return run(float(0));
    set_error("invalid dtype");
    return JFNK_ERR_ARG;
}

int jfnk_precond_apply(jfnk_ctx* c, jfnk_pc_kind pc, jfnk_dtype dt, const void* u, const void* r, void* z,
                       int32_t sweeps) {
    if (!c || !u || !r || !z || r == z || sweeps < 0) {
        set_error("invalid argument to jfnk_precond_apply");
        return JFNK_ERR_ARG;
    }
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        if (pc == JFNK_PC_PHYSICS) JFNK_HIP(op_frozen_nu<T>(c, (const T*)u, NUb<T>(c)));
        // div = null: r is read, never written
        return apply_pc<T>(c, pc, (const T*)u, (T*)r, nullptr, (T*)z, sweeps, TA<T>(c), EpsArgs());
    };
    if (dt == JFNK_F64) return run(double(0));
    if (dt == JFNK_F32) return run(float(0));
    set_error("invalid dtype");
    return JFNK_ERR_ARG;
}

static bool valid_gmres_opts(jfnk_ctx* c, const jfnk_gmres_opts* o) {
    if (!o || o->m < 1 || o->m > c->max_m || o->max_restarts < 1 || o->sweeps < 0 || o->jv < 0 || o->jv > 2) {
        set_error("invalid GMRES options (m must be in [1, max_m])");
        return false;
    }
    if (o->pc != JFNK_PC_NONE && o->pc != JFNK_PC_PHYSICS && o->pc != JFNK_PC_LEARNED) {
        set_error("unknown preconditioner kind");
        return false;
    }
    if (o->ortho != JFNK_ORTHO_CGS2 && o->ortho != JFNK_ORTHO_ONE_REDUCTION) {
        set_error("unknown orthogonalization");
        return false;
    }
    return true;
}

int jfnk_gmres(jfnk_ctx* c, jfnk_dtype dt, const void* u, const void* rhs, void* x, const jfnk_gmres_opts* o,
               jfnk_gmres_info* info) {
    if (!c || !u || !rhs || !x || !valid_gmres_opts(c, o)) {
        if (c && o) set_error(std::string("invalid argument to jfnk_gmres: ") + jfnk_last_error());
        return JFNK_ERR_ARG;
    }
    if (dt != JFNK_F64 && dt != JFNK_F32) {
        set_error("invalid dtype");
        return JFNK_ERR_ARG;
    }
    if (o->pc == JFNK_PC_LEARNED && (dt != JFNK_F32 || !c->net.ready)) {
        set_error("the learned preconditioner needs FP32 and parameters set (jfnk_net_set_params)");
        return JFNK_ERR_ARG;
    }
    jfnk_gmres_info local{};
    jfnk_gmres_info* gi = info ? info : &local;
    // the true residual ||rhs - J x|| of the returned x (the same Jv as the solve)
    auto finish = [&](auto zero_t, int rc) -> int {
        using T = decltype(zero_t);
        if (rc < 0) return rc;
        bool zero = false;
        int r2 = gmres_restart<T>(c, (const T*)u, (const T*)rhs, (const T*)x, *o, zero);
        if (r2) return r2;
        gi->res_true = c->hscal[S_BETA];
        return rc;
    };
    if (dt == JFNK_F64)
        return finish(double(0), krylov_solve<double>(c, (const double*)u, (const double*)rhs, (double*)x, *o, gi,
                                                      nullptr));
    return finish(float(0), krylov_solve<float>(c, (const float*)u, (const float*)rhs, (float*)x, *o, gi, nullptr));
}

int jfnk_norm(jfnk_ctx* c, jfnk_dtype dt, const void* x, int64_t n, double* out) {
    if (!c || !x || !out || n < 0) {
        set_error("invalid argument to jfnk_norm");
        return JFNK_ERR_ARG;
    }
    int rc = dt == JFNK_F64 ? norm2_to<double>(c, (const double*)x, n, sc(c, S_TMP))
                            : norm2_to<float>(c, (const float*)x, n, sc(c, S_TMP));
    if (rc) return rc;
    if ((rc = read_scalars(c, S_TMP, 1))) return rc;
    *out = std::sqrt(c->hscal[S_TMP]);
    return JFNK_OK;
}

int jfnk_newton_step(jfnk_ctx* c, const double* u_n, double* u, const jfnk_newton_opts* o, jfnk_newton_info* info) {
    if (!c || !u_n || !u || !o || !valid_gmres_opts(c, &o->gm) || o->max_newton < 0 ||
        (o->inner != JFNK_F64 && o->inner != JFNK_F32) || (o->gm.pc == JFNK_PC_LEARNED && o->inner != JFNK_F32)) {
        set_error(std::string("invalid argument to jfnk_newton_step"));
        return JFNK_ERR_ARG;
    }
    const long long n = c->n;
    hipStream_t s = c->stream;
    int rc;
    {
        TimedLaunch tl(c, KC_RESIDUAL);
        JFNK_HIP(op_F<double>(c, u_n, nullptr, c->f64, 1));
    }
    auto resid_norm = [&](double& out) -> int {
        {
            TimedLaunch tl(c, KC_RESIDUAL);
            JFNK_HIP(op_F<double>(c, u, c->f64, c->R64, 2));
        }
        int r2 = norm2_to<double>(c, c->R64, n, sc(c, S_TMP));
        if (r2) return r2;
        if ((r2 = read_scalars(c, S_TMP, 1))) return r2;
        out = std::sqrt(c->hscal[S_TMP]);
        return JFNK_OK;
    };
    double unorm;
    if ((rc = jfnk_norm(c, JFNK_F64, u_n, n, &unorm))) return rc;
    double rn;
    if ((rc = resid_norm(rn))) return rc;
    const double r0 = rn;
    const double tol = std::max(o->rtol * r0, o->atol_factor * (2.0 / c->prob.dt) * unorm);
    jfnk_newton_info inf{};
    inf.res0 = r0;
    const bool rec_sys = o->rec_r && o->rec_du && o->rec_count && !o->rec_krylov;
    struct RecGuard {
        jfnk_ctx* c;
        ~RecGuard() {
            c->rec_r = c->rec_du = nullptr;
            c->rec_count = nullptr;
            c->rec_cap = 0;
        }
    } rec_guard{c};
    if (o->rec_krylov && o->rec_r && o->rec_du && o->rec_count) {
        c->rec_r = o->rec_r;
        c->rec_du = o->rec_du;
        c->rec_cap = o->rec_cap;
        c->rec_count = o->rec_count;
    }
    double rprev = r0, eta = 0.5;
    bool converged = false;
    bool benched = false;   // the learned preconditioner fell short earlier in this step
    int k = 0;
    for (;; ++k) {
        if (!std::isfinite(rn)) {
            set_error("non-finite Newton residual");
            return JFNK_ERR_NONFINITE;
        }
        if (rn <= tol) {
            converged = true;
            break;
        }
        if (k >= o->max_newton) break;
        if (o->forcing == 0) {
            // Eisenstat-Walker choice 2 with the standard safeguards
            const double gamma = 0.9, alpha = 2.0, eta_max = 0.9;
            if (k == 0) {
                eta = 0.5;
            } else {
                double e = gamma * std::pow(rn / rprev, alpha);
                const double sg = gamma * std::pow(eta, alpha);
                if (sg > 0.1) e = std::max(e, sg);
                eta = std::min(e, eta_max);
            }
            eta = std::min(std::max(eta, 0.5 * tol / rn), eta_max);
        } else {
            eta = o->eta;
        }
        eta = std::max(eta, o->eta_floor);
        jfnk_gmres_opts go = o->gm;
        go.tol = eta;
        jfnk_gmres_info gi{};
        if (o->inner == JFNK_F64) {
            JFNK_HIP(launch_cast<double, double>(c->b64, c->R64, n, -1.0, s));
            rc = krylov_solve<double>(c, u, c->b64, c->x64, go, &gi, nullptr);
            if (rc < 0) return rc;
            if (rec_sys && *o->rec_count < o->rec_cap) {
                const long long off = (long long)(*o->rec_count) * n;
                JFNK_HIP(launch_cast<float, double>(o->rec_r + off, c->b64, n, 1.0, s));
                JFNK_HIP(launch_cast<float, double>(o->rec_du + off, c->x64, n, 1.0, s));
                ++*o->rec_count;
            }
            JFNK_HIP(launch_add_to64<double>(u, c->x64, n, s));
        } else {
            JFNK_HIP(launch_cast<float, double>(c->u32, u, n, 1.0, s));
            JFNK_HIP(launch_cast<float, double>(c->b32, c->R64, n, -1.0, s));
            rc = krylov_solve<float>(c, c->u32, c->b32, c->x32, go, &gi, &inf.gmres_iters_total, &benched);
            if (go.pc == JFNK_PC_LEARNED && gi.fallback) inf.fallbacks++;
            if (rc < 0) return rc;
            if (rec_sys && *o->rec_count < o->rec_cap) {
                const long long off = (long long)(*o->rec_count) * n;
                JFNK_HIP(hipMemcpyAsync(o->rec_r + off, c->b32, n * sizeof(float), hipMemcpyDeviceToDevice, s));
                JFNK_HIP(hipMemcpyAsync(o->rec_du + off, c->x32, n * sizeof(float), hipMemcpyDeviceToDevice, s));
                ++*o->rec_count;
            }
            JFNK_HIP(launch_add_to64<float>(u, c->x32, n, s));
        }
        inf.gmres_iters_total += gi.iters;
        rprev = rn;
        if ((rc = resid_norm(rn))) return rc;
    }
    inf.newton_iters = k;
    inf.converged = converged ? 1 : 0;
    inf.res_final = rn;
    if (info) *info = inf;
    return converged ? JFNK_OK : JFNK_NOT_CONVERGED;
}

int jfnk_nlpc_residual(jfnk_ctx* c, const double* u, const double* f, double* out, int32_t sweeps) {
    if (!c || !u || !f || !out || out == u || out == f || sweeps < 0) {
        set_error("invalid argument to jfnk_nlpc_residual");
        return JFNK_ERR_ARG;
    }
    JFNK_HIP(hipMemcpyAsync(c->f64, f, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return rtilde64(c, u, c->R64, out, c->t64a, sweeps);
}

int jfnk_nlpc_step(jfnk_ctx* c, const double* u_n, double* u, const jfnk_newton_opts* o, int32_t method,
                   jfnk_newton_info* info) {
    if (!c || !u_n || !u || !o || (method != 0 && method != 1) || o->max_newton < 0 || o->gm.sweeps < 0 ||
        (method == 1 && (o->gm.m < 1 || o->gm.m > c->max_m || o->gm.max_restarts < 1))) {
        set_error("invalid argument to jfnk_nlpc_step");
        return JFNK_ERR_ARG;
    }
    const long long n = c->n;
    hipStream_t s = c->stream;
    int rc;
    c->nl_sweeps = o->gm.sweeps;
    {
        TimedLaunch tl(c, KC_RESIDUAL);
        JFNK_HIP(op_F<double>(c, u_n, nullptr, c->f64, 1));
    }
    auto norm_of = [&](const double* x, double& out) -> int {
        int r2 = norm2_to<double>(c, x, n, sc(c, S_TMP));
        if (r2) return r2;
        if ((r2 = read_scalars(c, S_TMP, 1))) return r2;
        out = std::sqrt(c->hscal[S_TMP]);
        return JFNK_OK;
    };
    auto resid_norm = [&](double& out) -> int {
        {
            TimedLaunch tl(c, KC_RESIDUAL);
            JFNK_HIP(op_F<double>(c, u, c->f64, c->R64, 2));
        }
        return norm_of(c->R64, out);
    };
    // R~(u) = P^{-1}(u) R(u) from the residual already in R64
    auto rtilde_norm = [&](double* dst, double* scratch, double& out) -> int {
        JFNK_HIP(op_frozen_nu<double>(c, u, NUb<double>(c)));
        int r2 = apply_pc<double>(c, JFNK_PC_PHYSICS, u, c->R64, nullptr, dst, o->gm.sweeps, scratch, EpsArgs());
        if (r2) return r2;
        return norm_of(dst, out);
    };
    double unorm, rn;
    if ((rc = norm_of(u_n, unorm))) return rc;
    if ((rc = resid_norm(rn))) return rc;
    const double r0 = rn;
    const double tol = std::max(o->rtol * r0, o->atol_factor * (2.0 / c->prob.dt) * unorm);
    jfnk_newton_info inf{};
    inf.res0 = r0;
    bool converged = false;
    int k = 0;
    double rt = 0.0, rt_prev = 0.0, tol_t = 0.0, eta = 0.5;
    if (method == 1) {
        if ((rc = rtilde_norm(c->nl64, c->nls64, rt))) return rc;
        tol_t = o->rtol * rt;
        rt_prev = rt;
    }
    for (;; ++k) {
        if (!std::isfinite(rn)) {
            set_error("non-finite residual in the nonlinear preconditioning");
            return JFNK_ERR_NONFINITE;
        }
        if (rn <= tol) {
            converged = true;
            break;
        }
        if (k >= o->max_newton) break;
        if (method == 0) {
            // fixed point u <- u - P^{-1}(u) R(u)
            double dummy;
            if ((rc = rtilde_norm(c->t64a, c->t64b, dummy))) return rc;
            JFNK_HIP(launch_lincomb<double>(u, u, c->t64a, n, 1.0, -1.0, s));
        } else {
            // inexact Newton on R~ with Eisenstat-Walker forcing on ||R~||
            if (o->forcing == 0) {
                const double gamma = 0.9, alpha = 2.0, eta_max = 0.9;
                if (k == 0) {
                    eta = 0.5;
                } else {
                    double e = gamma * std::pow(rt / rt_prev, alpha);
                    const double sg = gamma * std::pow(eta, alpha);
                    if (sg > 0.1) e = std::max(e, sg);
                    eta = std::min(e, eta_max);
                }
                eta = std::min(std::max(eta, 0.5 * tol_t / rt), eta_max);
            } else {
                eta = o->eta;
            }
            eta = std::max(eta, o->eta_floor);
            jfnk_gmres_opts go = o->gm;
            go.tol = eta;
            go.pc = JFNK_PC_NONE;
            go.jv = kJvNlpc;
            jfnk_gmres_info gi{};
            JFNK_HIP(launch_cast<double, double>(c->b64, c->nl64, n, -1.0, s));
            rc = gmres_impl<double>(c, u, c->b64, c->x64, go, &gi);
            if (rc < 0) return rc;
            inf.gmres_iters_total += gi.iters;
            JFNK_HIP(launch_add_to64<double>(u, c->x64, n, s));
        }
        if ((rc = resid_norm(rn))) return rc;
        if (method == 1) {
            rt_prev = rt;
            if ((rc = rtilde_norm(c->nl64, c->nls64, rt))) return rc;
        }
    }
    inf.newton_iters = k;
    inf.converged = converged ? 1 : 0;
    inf.res_final = rn;
    if (info) *info = inf;
    return converged ? JFNK_OK : JFNK_NOT_CONVERGED;
}

int jfnk_set_variant(jfnk_ctx* c, int32_t stage, int32_t dtype, int32_t variant) {
    if (!c) {
        set_error("null context");
        return JFNK_ERR_ARG;
    }
    if (c->geo.dim == 3) {
        // 3D: only the FP32 Jv has two forms
        if (stage != 1 || dtype != JFNK_F32 || (variant != 6 && variant != 7)) {
            set_error("3D contexts take variant 6 (two-pass) or 7 (single-pass) of the FP32 Jv");
            return JFNK_ERR_ARG;
        }
        c->jv3_single = variant == 7 ? 1 : 0;
        return JFNK_OK;
    }
    if (stage < 0 || stage > 2 || (dtype != JFNK_F64 && dtype != JFNK_F32) || variant < 0 ||
        variant > (stage < 2 ? 5 : 2) || (stage == 1 && dtype == JFNK_F64 && variant == 2)) {
        set_error("invalid stage, dtype or variant");
        return JFNK_ERR_ARG;
    }
    c->tune[stage * 2 + (dtype == JFNK_F32 ? 1 : 0)] = variant;
    return JFNK_OK;
}

int jfnk_tune(jfnk_ctx* c, int32_t* tile_rows) {
    if (!c) {
        set_error("null context");
        return JFNK_ERR_ARG;
    }
    if (c->geo.dim == 3) {               // the 3D kernels have a single launch shape
        if (tile_rows)
            for (int k = 0; k < 6; ++k) tile_rows[k] = 0;
        return JFNK_OK;
    }
    hipEvent_t e0, e1;
    JFNK_HIP(hipEventCreate(&e0));
    JFNK_HIP(hipEventCreate(&e1));
    int rc = tune_precision<double>(c, e0, e1);
    if (!rc) rc = tune_precision<float>(c, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (tile_rows)
        for (int k = 0; k < 6; ++k) tile_rows[k] = tile_tz(c->tune[k]);
    return JFNK_OK;
}

int jfnk_timing_enable(jfnk_ctx* c, int32_t enable) {
    if (!c) {
        set_error("null context");
        return JFNK_ERR_ARG;
    }
    resolve_timing(c);
    for (int k = 0; k < KC_COUNT; ++k) {
        c->timing.ms[k] = 0.0;
        c->timing.launches[k] = 0;
        c->timing.bytes[k] = 0.0;
    }
    c->timing.on = enable != 0;
    c->timing.mask = enable < 0 ? ~0u : (unsigned)enable;
    return JFNK_OK;
}

int jfnk_timing_read(jfnk_ctx* c, int32_t cls, double* total_ms, int64_t* launches, double* bytes) {
    if (!c || cls < 0 || cls >= KC_COUNT) {
        set_error("invalid argument to jfnk_timing_read");
        return JFNK_ERR_ARG;
    }
    resolve_timing(c);
    if (total_ms) *total_ms = c->timing.ms[cls];
    if (launches) *launches = c->timing.launches[cls];
    if (bytes) *bytes = c->timing.bytes[cls];
    return JFNK_OK;
}


int jfnk_net_init(jfnk_ctx* c, const int32_t* dilations, int64_t* n_params) {
    if (!c) {
        set_error("null context");
        return JFNK_ERR_ARG;
    }
    NetBuffers& nb = c->net;
    const int dim = c->prob.dim;
    for (int l = 0; l < 4; ++l) {
        const int d = dilations ? dilations[l] : 1;
        if (d < 1 || d > 8 || (dim == 3 && d != 1)) {
            set_error(dim == 3 ? "the 3D network has dilation 1" : "dilations must be in [1, 8]");
            return JFNK_ERR_ARG;
        }
        nb.dil[l] = d;
    }
    const int taps = dim == 3 ? 27 : 9;
    const int np = dim == 3 ? net3_param_count(c->nf) : net_param_count(c->nf);
    if (n_params) *n_params = np;
    if (nb.theta) return JFNK_OK;
    nb.dim = dim;
    const long long npts = c->geo.npts;
    const long long tiles = dim == 3 ? net3_wgrad_tiles(c->geo.nx, c->geo.ny, c->geo.nz)
                                     : (long long)((c->geo.nx + 63) / 64) * ((c->geo.nz + 3) / 4);
    nb.nparam = np;
#define NALLOC(ptr, count)                                                   \
    do {                                                                     \
        hipError_t e_ = hipMalloc((void**)&(ptr), sizeof(*(ptr)) * (count)); \
        if (e_ != hipSuccess) return hip_fail(e_, "hipMalloc " #ptr);        \
    } while (0)
    NALLOC(nb.theta, np);
    NALLOC(nb.grad, np);
    NALLOC(nb.m, np);
    NALLOC(nb.v, np);
    NALLOC(nb.wt, np);
    NALLOC(nb.wbf, 4 * taps * 16 * 16);
    NALLOC(nb.s, 16);
    NALLOC(nb.partials, 8192);
    NALLOC(nb.scal, 4);
    NALLOC(nb.loss, 4);
    NALLOC(nb.act, 4 * 16 * npts);
    NALLOC(nb.pre, 4 * 16 * npts);
    NALLOC(nb.a0, (long long)c->nf * npts);
    NALLOC(nb.z, (long long)c->nf * npts);
    NALLOC(nb.g0, 16 * npts);
    NALLOC(nb.g1, 16 * npts);
    NALLOC(nb.wpart, tiles * (16 * 16 * taps + 16));
    NALLOC(nb.abf, 2 * 16 * npts);
#undef NALLOC
    JFNK_HIP(hipMemsetAsync(nb.theta, 0, np * sizeof(float), c->stream));
    JFNK_HIP(hipMemsetAsync(nb.m, 0, np * sizeof(float), c->stream));
    JFNK_HIP(hipMemsetAsync(nb.v, 0, np * sizeof(float), c->stream));
    JFNK_HIP(hipStreamSynchronize(c->stream));
    nb.adam_t = 0;
    return JFNK_OK;
}

static hipError_t net_prep(jfnk_ctx* c) {
    return c->net.dim == 3 ? net3_prep_weights(c->net, c->nf, c->stream) : net_prep_weights(c->net, c->nf, c->stream);
}

static bool net_ok(jfnk_ctx* c) {
    if (!c || !c->net.theta) {
        set_error("call jfnk_net_init first");
        return false;
    }
    return true;
}

int jfnk_net_set_params(jfnk_ctx* c, const float* theta, int64_t n) {
    if (!net_ok(c) || !theta || n != c->net.nparam) {
        if (c && c->net.theta) set_error("parameter count mismatch");
        return JFNK_ERR_ARG;
    }
    JFNK_HIP(hipMemcpyAsync(c->net.theta, theta, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    JFNK_HIP(hipMemsetAsync(c->net.m, 0, n * sizeof(float), c->stream));
    JFNK_HIP(hipMemsetAsync(c->net.v, 0, n * sizeof(float), c->stream));
    c->net.adam_t = 0;
    JFNK_HIP(net_prep(c));
    JFNK_HIP(hipStreamSynchronize(c->stream));
    c->net.ready = true;
    return JFNK_OK;
}

int jfnk_net_get_params(jfnk_ctx* c, float* theta, int64_t n) {
    if (!net_ok(c) || !theta || n != c->net.nparam) return JFNK_ERR_ARG;
    JFNK_HIP(hipMemcpyAsync(theta, c->net.theta, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    JFNK_HIP(hipStreamSynchronize(c->stream));
    return JFNK_OK;
}

int jfnk_net_apply(jfnk_ctx* c, int32_t bf16, const float* r, float* z) {
    if (!net_ok(c) || !r || !z || !c->net.ready) {
        set_error("invalid argument to jfnk_net_apply (parameters set?)");
        return JFNK_ERR_ARG;
    }
    TimedLaunch tl(c, KC_NET, 2.0 * c->net.nparam * c->geo.npts);
    JFNK_HIP(net_run(c, r, z, bf16 != 0));
    return JFNK_OK;
}

// Loss and gradient over a batch of pairs on the grid nx x ny x nz (the context's
// or a crop of it, see jfnk_net_train_step).
static int net_batch_grad(jfnk_ctx* c, const float* r, const float* du, int32_t batch, double* loss, int nx, int ny,
                          int nz) {
    NetBuffers& nb = c->net;
    const float hdt = (float)(0.5 * c->prob.dt);
    const long long nvec = (long long)c->nf * nx * ny * nz;
    for (int b = 0; b < batch; ++b) {
        const float* rb = r + (long long)b * nvec;
        const float* db = du + (long long)b * nvec;
        if (nb.dim == 3)
            JFNK_HIP(net3_pair_grad(nb, nx, ny, nz, c->nf, hdt, rb, db, 1.0 / batch, b == 0, c->stream));
        else
            JFNK_HIP(net_pair_grad(nb, nx, nz, c->nf, hdt, rb, db, 1.0 / batch, b == 0, c->geo, c->stream));
    }
    if (loss) {
        JFNK_HIP(hipMemcpyAsync(loss, nb.loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        JFNK_HIP(hipStreamSynchronize(c->stream));
    }
    return JFNK_OK;
}

int jfnk_net_set_loss(jfnk_ctx* c, int32_t kind) {
    if (!net_ok(c) || (kind != JFNK_NET_LOSS_SOLUTION && kind != JFNK_NET_LOSS_REST_JACOBIAN)) {
        set_error("invalid argument to jfnk_net_set_loss");
        return JFNK_ERR_ARG;
    }
    if (kind == JFNK_NET_LOSS_REST_JACOBIAN && (c->prob.energy_test || c->prob.dim != 2 || c->prob.dd_p != 2)) {
        set_error("the rest-Jacobian loss is available for 2D problems with energy_test = 0 and dd_p = 2");
        return JFNK_ERR_ARG;
    }
    c->net.loss_kind = kind;
    return JFNK_OK;
}

int jfnk_net_loss_grad(jfnk_ctx* c, const float* r, const float* du, int32_t batch, double* loss, float* grad) {
    if (!net_ok(c) || !r || !du || batch < 1 || !c->net.ready) {
        set_error("invalid argument to jfnk_net_loss_grad");
        return JFNK_ERR_ARG;
    }
    int rc = net_batch_grad(c, r, du, batch, loss, c->geo.nx, c->geo.ny, c->geo.nz);
    if (rc) return rc;
    if (grad) {
        JFNK_HIP(hipMemcpyAsync(grad, c->net.grad, c->net.nparam * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        JFNK_HIP(hipStreamSynchronize(c->stream));
    }
    return JFNK_OK;
}

int jfnk_net_train_step(jfnk_ctx* c, const float* r, const float* du, int32_t batch, const int32_t* crop_dims,
                        float lr, double* loss) {
    if (!net_ok(c) || !r || !du || batch < 1 || !(lr > 0) || !c->net.ready) {
        set_error("invalid argument to jfnk_net_train_step");
        return JFNK_ERR_ARG;
    }
    int nx = c->geo.nx, ny = c->geo.ny, nz = c->geo.nz;
    if (crop_dims) {
        nx = crop_dims[0];
        ny = crop_dims[1];
        nz = crop_dims[2];
        const bool whole = nx == c->geo.nx && ny == c->geo.ny && nz == c->geo.nz;
        if (nx < 1 || ny < 1 || nz < 1 || nx > c->geo.nx || ny > c->geo.ny || nz > c->geo.nz ||
            (c->prob.dim == 2 && ny != 1) || (!whole && c->net.loss_kind != NET_LOSS_SOLUTION)) {
            set_error("invalid crop_dims for jfnk_net_train_step (within the grid, ny = 1 in 2D, solution loss)");
            return JFNK_ERR_ARG;
        }
    }
    int rc = net_batch_grad(c, r, du, batch, loss, nx, ny, nz);
    if (rc) return rc;
    c->net.adam_t++;
    JFNK_HIP(net_adam(c->net, c->net.nparam, c->net.adam_t, lr, c->stream));
    JFNK_HIP(net_prep(c));
    return JFNK_OK;
}

}  // extern "C"

// ---- Jv without a context, allocating nothing ------------------------------
// The device memory this entry point needs beyond its inputs and output (the
// background profiles p_bar, dp_bar/dz of both precisions, the partial sums and
// scalars of the finite-difference step) is a fixed file-scope array, one copy
// per GPU, held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's name
// in host code is not a device address).
constexpr int kNoAllocMaxNz = 4096;
constexpr int kNoAllocScalars = 8;
constexpr long long kNoAllocDoubles =
    2LL * kNoAllocMaxNz + kNoAllocMaxNz /* two float profiles */ + kMaxPartials + kNoAllocScalars;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array (looked up once per device)
int scratch_ptr(double** out) {
    int dev = 0;
    JFNK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index out of range for the no-allocation scratch table");
        return JFNK_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        JFNK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the scratch array");
            return JFNK_ERR_HIP;
        }
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return JFNK_OK;
}
}  // namespace

extern "C" int jfnk_jv_noalloc(const jfnk_problem* p, jfnk_dtype dt, jfnk_jv_mode mode, const void* u, const void* v,
                               double eps, void* Jv, void* hip_stream) {
    std::string why;
    if (!p || !u || !v || !Jv || (mode != JFNK_JV_STABLE && mode != JFNK_JV_ANALYTIC) ||
        (dt != JFNK_F64 && dt != JFNK_F32) || !valid_problem(p, why)) {
        set_error("invalid argument to jfnk_jv_noalloc" + (why.empty() ? std::string() : ": " + why));
        return JFNK_ERR_ARG;
    }
    if (p->nz > kNoAllocMaxNz) {
        set_error("jfnk_jv_noalloc: nz exceeds " + std::to_string(kNoAllocMaxNz));
        return JFNK_ERR_ARG;
    }
    if (p->dim == 3 && (dt != JFNK_F32 || p->dd_p != 2)) {
        set_error("jfnk_jv_noalloc: 3D problems take the FP32 single-pass Jv (dd_p = 2) only");
        return JFNK_ERR_ARG;
    }
    double* sp = nullptr;
    int rc = scratch_ptr(&sp);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    Geo g;
    fill_geo(*p, g);
    double* pb64 = sp;
    double* dpb64 = sp + kNoAllocMaxNz;
    float* pb32 = (float*)(sp + 2 * kNoAllocMaxNz);
    float* dpb32 = pb32 + kNoAllocMaxNz;
    double* partials = sp + 3 * kNoAllocMaxNz;
    double* scal = partials + kMaxPartials;   // ||u||^2, ||v||^2, eps
    g.pbar64 = pb64;
    g.dpbar64 = dpb64;
    g.sflux64 = nullptr;                      // the surface source does not enter Jv
    g.pbar32 = pb32;
    g.dpbar32 = dpb32;
    g.sflux32 = nullptr;
    hipLaunchKernelGGL(k_background, dim3((g.nz + 255) / 256), dim3(256), 0, st, g, *p, pb64, dpb64, (double*)nullptr,
                       pb32, dpb32, (float*)nullptr);
    JFNK_HIP(hipGetLastError());
    const long long n = (long long)(p->dim == 3 ? 5 : 4) * g.npts;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        const double* edev = nullptr;
        if (mode == JFNK_JV_STABLE && !(eps > 0)) {
            const int nb = red_blocks(n);
            JFNK_HIP(launch_norm2_partial<T>((const T*)u, n, partials, nb, st));
            JFNK_HIP(launch_reduce_partials(partials, nb, 1, 1, scal, 0, st));
            JFNK_HIP(launch_norm2_partial<T>((const T*)v, n, partials, nb, st));
            JFNK_HIP(launch_reduce_partials(partials, nb, 1, 1, scal + 1, 0, st));
            JFNK_HIP(launch_fd_eps(scal, scal + 1, std::sqrt(eps_mach<T>()), std::sqrt((double)n), scal + 2, st));
            edev = scal + 2;
        }
        const double e = mode == JFNK_JV_ANALYTIC ? 0.0 : eps;
        if constexpr (std::is_same<T, float>::value) {
            if (g.dim == 3) {
                JFNK_HIP(launch3_jv_fused(g, (const float*)u, (const float*)v, e, edev, (float*)Jv, st));
                return JFNK_OK;
            }
        }
        JFNK_HIP(launch_jv<T>(g, (const T*)u, (const T*)v, e, edev, (T*)Jv, st, 1));
        return JFNK_OK;
    };
    return dt == JFNK_F64 ? run(double(0)) : run(float(0));
}
