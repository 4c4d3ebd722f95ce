// Internal declarations of the JFNK HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/jfnk.h"

namespace jfnk {

// Kernel-side view of a problem: constants and device pointers, passed by value.
// FP32 copies of the constants the FP32 kernels use, rounded once on the host
// (kernel-argument scalars rather than per-thread conversions)
struct GeoF {
    float idx, idy, idz, two_dt, theta0, g_theta0, kappa, kappa_cp, beta;
    float smag_s2;   // (float)smag * sqrt2, the Smagorinsky nu per unit |S|
    float inv_pr, dd_ah, dd_av, dd_ch, dd_cv, dd_b, dd_delta;
};

struct Geo {
    int dim, nx, ny, nz;
    int W = 2;                  // half-width of the derivative stencil (2: p = 2, 4: p = 3)
    long long npts;
    int bcl, bcv;               // lateral / vertical boundary kind
    double dx, dy, dz;
    double idx, idy, idz;       // inverse spacings
    double two_dt;              // 2 / dt
    double theta0, g_theta0;    // theta0, g / theta0
    double kappa, kappa_cp;     // kappa, kappa * cp (energy-test coefficient)
    double beta;
    int closure;
    double smag;                // (cs * Delta)^2
    double inv_pr;              // 1 / Pr_t
    double k_m, k_h;
    // anisotropic coefficients (closure 3, 2D): K_m = dd_ah |S|, K_M = dd_av |S|,
    // l = min(dd_b |S|, dd_delta) (dd_b = 0: l = dd_delta), K_h = K_m + dd_ch l |S|,
    // K_H = K_M + dd_cv l |S|; |S| = nu_tau * dd_inv_nu
    double dd_ah, dd_av, dd_ch, dd_cv, dd_b, dd_delta, dd_inv_nu;
    int convection, energy_test;
    const double* pbar64;       // p_bar(z), [nz]
    const double* dpbar64;      // dp_bar/dz(z), [nz]
    const double* sflux64;      // Q(x, y) / dz, [ny * nx]
    const float* pbar32;
    const float* dpbar32;
    const float* sflux32;
    GeoF f;
};

template <typename T> struct Bg;
template <> struct Bg<double> {
    static __device__ __forceinline__ const double* pbar(const Geo& g) { return g.pbar64; }
    static __device__ __forceinline__ const double* dpbar(const Geo& g) { return g.dpbar64; }
    static __device__ __forceinline__ const double* sflux(const Geo& g) { return g.sflux64; }
};
template <> struct Bg<float> {
    static __device__ __forceinline__ const float* pbar(const Geo& g) { return g.pbar32; }
    static __device__ __forceinline__ const float* dpbar(const Geo& g) { return g.dpbar32; }
    static __device__ __forceinline__ const float* sflux(const Geo& g) { return g.sflux32; }
};

// Arguments of the FP64 Givens step of GMRES column j (device pointers;
// host = optional pinned mirror receiving (||w||, |g_{j+1}|)).
struct GivensArgs {
    double* H = nullptr;
    double* Hraw = nullptr;
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;
    const double* h1 = nullptr;
    const double* h2 = nullptr;
    double* wnorm = nullptr;
    double* res_est = nullptr;
    double* host = nullptr;
    int j = 0;
    int m = 0;
};

// Finite-difference step of the Jacobian-vector product from squared norms:
// eps = sqrt(eps_mach) max(||u||, sqrt(N)) / ||v||  (0 when v = 0).
struct EpsArgs {
    double* partials = nullptr;   // null: no norm requested
    const double* unorm2 = nullptr;
    double* vnorm2 = nullptr;
    double* eps = nullptr;
    double sqrt_eps = 0.0;
    double sqrt_n = 0.0;
};

// per-instance scalar block of a batch (doubles)
constexpr int S_STRIDE = 16;
enum { SB_UNORM2 = 0, SB_VNORM2 = 1, SB_EPS = 2, SB_WNORM = 3, SB_RES = 4, SB_BETA = 5, SB_SQRTN = 6 };

enum CgsMode { CGS_DOT = 0, CGS_UPD_DOT = 1, CGS_UPD_NORM = 2 };

enum KernelClass { KC_JV = 0, KC_RESIDUAL = 1, KC_PC = 2, KC_ARNOLDI = 3, KC_VEC = 4, KC_NET = 5, KC_COUNT = 6 };

constexpr int kMaxPartials = 2048;   // blocks of a reduction grid
constexpr int kMaxDots = 64;         // vectors per fused dot pass (>= max_m + 1)

// Event pairs recorded around kernel launches of each class while timing is on;
// elapsed times are resolved lazily (no host synchronisation per launch).
struct Timing {
    bool on = false;
    unsigned mask = 0;                      // classes recorded (bit k: class k)
    std::vector<hipEvent_t> ev[KC_COUNT];   // 2 per launch
    int used[KC_COUNT] = {0};
    double ms[KC_COUNT] = {0};
    long long launches[KC_COUNT] = {0};
    double bytes[KC_COUNT] = {0};           // algorithmic HBM bytes of the timed launches
};

// Workspace of the learned preconditioner (allocated by jfnk_net_init).
struct NetBuffers {
    float* theta = nullptr;          // FP32 master parameters
    float* grad = nullptr;
    float* m = nullptr;              // Adam moments
    float* v = nullptr;
    float* wt = nullptr;             // transposed, flipped weights (backward data)
    unsigned short* wbf = nullptr;   // bf16 weights [layer][tap][co][ci], 16 x 16 padded (9 or 27 taps)
    float* s = nullptr;              // per-field scales
    double* partials = nullptr;
    double* scal = nullptr;
    double* loss = nullptr;
    float* act = nullptr;            // 4 x 16 x npts post-activations
    float* pre = nullptr;            // 4 x 16 x npts pre-activations
    float* a0 = nullptr;             // nf x npts scaled input
    float* z = nullptr;              // nf x npts output
    float* g0 = nullptr;             // 16 x npts gradients
    float* g1 = nullptr;
    float* wpart = nullptr;          // per-tile weight-gradient partials
    unsigned short* abf = nullptr;   // 2 x npts x 16 bf16 activations, pixel-major (channel innermost)
    int nparam = 0;
    int adam_t = 0;
    int dil[4] = {1, 1, 1, 1};       // per-layer dilation of the 3x3 kernels
    int loss_kind = 0;               // NET_LOSS_SOLUTION or NET_LOSS_REST_JACOBIAN
    int dim = 2;                     // 2: 3x3 kernels, 3: 3x3x3 kernels
    bool ready = false;              // parameters set
};
enum { NET_LOSS_SOLUTION = 0, NET_LOSS_REST_JACOBIAN = 1 };

int net_param_count(int nf);
hipError_t net_prep_weights(const NetBuffers& nb, int nf, hipStream_t s);
// BF16 path only, may be null: ea, the FD step of the next Jv formed from z;
// rpart, rnblk partial sums of r^2 over all fields left by r's producer
hipError_t net_apply(const NetBuffers& nb, int nx, int nz, int nf, float half_dt, const float* r, float* z,
                     bool bf16, hipStream_t st, const EpsArgs* ea = nullptr, const double* rpart = nullptr,
                     int rnblk = 0);
hipError_t net_pair_grad(const NetBuffers& nb, int nx, int nz, int nf, float half_dt, const float* r,
                         const float* du, double inv_batch, bool first_pair, const Geo& geo, hipStream_t st);
hipError_t net_adam(const NetBuffers& nb, int n, int t, float lr, hipStream_t st);
hipError_t net_field_scale(const float* r, long long np, int nf, double* partials, float* s, hipStream_t st);
hipError_t net_field_sumsq(const float* r, long long np, int nf, double* partials, hipStream_t st);
int net_sumsq_blocks(long long np);
hipError_t net_scale_source(const float* r, long long np, int nf, const double* rpart, int rnblk, double* partials,
                            float* s, int fuse_limit, const double** part, int* nblk, int* nsets, hipStream_t st);
hipError_t net_solution_loss(const NetBuffers& nb, long long np, int nf, const float* du, double inv_batch,
                             bool first_pair, hipStream_t st);
hipError_t net_cast_scaled(const float* r, long long np, int nf, const float* s, float* out, hipStream_t st);
hipError_t net_wgrad_finish(const float* partials, int nblk, int cnt, float* grad, bool accumulate, hipStream_t st);
// 3D network (3 x 3 x 3 kernels, dilation 1)
int net3_param_count(int nf);
long long net3_wgrad_tiles(int nx, int ny, int nz);
hipError_t net3_prep_weights(const NetBuffers& nb, int nf, hipStream_t s);
hipError_t net3_apply(const NetBuffers& nb, int nx, int ny, int nz, int nf, float half_dt, const float* r, float* z,
                      bool bf16, hipStream_t st, const EpsArgs* ea = nullptr, const double* rpart = nullptr,
                      int rnblk = 0);
hipError_t net3_pair_grad(const NetBuffers& nb, int nx, int ny, int nz, int nf, float half_dt, const float* r,
                          const float* du, double inv_batch, bool first_pair, hipStream_t st);

}  // namespace jfnk

struct jfnk_ctx {
    jfnk_problem prob;
    jfnk::Geo geo;
    int device = 0;
    hipStream_t stream = nullptr;
    int max_m = 0;
    int nf = 0;
    long long n = 0;            // nf * npts
    // Krylov bases
    double* V64 = nullptr;      // (max_m + 1) * n
    double* Z64 = nullptr;      // max_m * n
    float* V32 = nullptr;
    float* Z32 = nullptr;
    // FP64 temporaries
    double* f64 = nullptr;      // f(u^n)
    double* R64 = nullptr;      // residual
    double* nl64 = nullptr;     // R~(u) of the nonlinear preconditioning (cached for its FD Jacobian)
    double* nls64 = nullptr;    // preconditioner scratch of the nonlinear preconditioning
    int nl_sweeps = 2;
    double* t64a = nullptr;
    double* t64b = nullptr;
    double* b64 = nullptr;      // Newton right-hand side -R
    double* x64 = nullptr;      // Newton correction
    double* nu64 = nullptr;     // frozen eddy viscosity on the ring-2 extended grid
    double* d64 = nullptr;      // 3D: stress / heat-flux buffer [9][ext]
    float* d32 = nullptr;
    // FP32 temporaries
    float* u32 = nullptr;
    float* b32 = nullptr;
    float* x32 = nullptr;
    float* t32a = nullptr;
    float* t32b = nullptr;
    float* nu32 = nullptr;
    // background
    double* bg64 = nullptr;     // pbar | dpbar | sflux
    float* bg32 = nullptr;
    // reductions and small device state
    double* partials = nullptr; // kMaxPartials * kMaxDots
    double* epart = nullptr;    // per-block partials of the FD-step norm
    double* qpart = nullptr;    // per-block partials of ||q~_{j+1}||^2 from the Arnoldi update pass
    double* dscal = nullptr;    // device scalars (see solver)
    double* hscal = nullptr;    // pinned host mirror
    hipEvent_t slot_ev[4] = {nullptr, nullptr, nullptr, nullptr};  // GMRES result slots in flight
    jfnk::Timing timing;
    jfnk::NetBuffers net;
    int fallbacks = 0;
    // physics-based preconditioner as the judge of the learned one: mean log
    // residual reduction per Krylov iteration of the last physics-preconditioned
    // solve of this context (0: none on record), the bound a running learned
    // solve is held to (0: none) and whether it fell short
    double judge_rate = 0.0;
    double judge_active = 0.0;
    bool judged_out = false;
    // tile variant per stencil stage, chosen by jfnk_tune (index: stage * 2 + (FP32 ? 1 : 0);
    // stages 0 residual / F, 1 Jv, 2 preconditioner sweep)
    int tune[6] = {1, 1, 1, 1, 1, 1};
    // 3D FP32 Jv: the single-pass kernel (1) or the two-pass form with the
    // stress / heat-flux buffer (0)
    int jv3_single = 1;
    // Krylov-pair recording (J z_j, z_j) during FP32 solves
    float* rec_r = nullptr;
    float* rec_du = nullptr;
    int rec_cap = 0;
    int* rec_count = nullptr;
};

namespace jfnk {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define JFNK_HIP(...)                                                     \
    do {                                                                  \
        hipError_t e_ = (__VA_ARGS__);                                    \
        if (e_ != hipSuccess) return ::jfnk::hip_fail(e_, #__VA_ARGS__);  \
    } while (0)

// ---- kernel launchers (stencil.hip) ----
// out = F(u) (what 0), 2u/dt + F(u) (what 1), 2u/dt - F(u) - f (what 2)
// var: tile variant chosen by the autotuner (tile height 4 << var)
int tile_tz(int variant);
// device geometry and coefficients of a problem (grid, boundaries, constants, closure)
void fill_geo(const jfnk_problem& p, Geo& g);
template <typename T>
hipError_t launch_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, hipStream_t s, int var = 1);
// Jv = 2v/dt - [F(u + eps v) - F(u)]/eps, expanded; eps read from *eps_dev if non-null
template <typename T>
hipError_t launch_jv(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, T* jv,
                     hipStream_t s, int var = 1);
// frozen eddy viscosity nu(u) at the grid points
template <typename T>
hipError_t launch_frozen_nu(const Geo& g, const T* u, T* nu, hipStream_t s);
// one Jacobi sweep of the physics preconditioner: zout = zin + (r - P zin)/d
// (zin == nullptr: zin = r/d)
template <typename T>
hipError_t launch_pc_sweep(const Geo& g, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                           const EpsArgs& ea, hipStream_t s, int var = 1);
// z = v / d with v = V_j / *div written back into V_j when div != null; the norm of
// z (for the FD step) when ea.partials != null
template <typename T>
hipError_t launch_pc_diag(const Geo& g, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea,
                          hipStream_t s);

// ---- 3D kernels (stencil3d.hip); dbuf: [9][nz+4][ny+4][nx+4] scratch ----
template <typename T>
hipError_t launch3_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, T* dbuf, hipStream_t s);
template <typename T>
hipError_t launch3_jv(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, T* out, T* dbuf,
                      hipStream_t s);
// the FP32 Jv in one z-marching launch (no intermediate buffer)
hipError_t launch3_jv_fused(const Geo& g, const float* u, const float* v, double eps, const double* eps_dev,
                            float* out, hipStream_t s);
template <typename T>
hipError_t launch3_frozen_nu(const Geo& g, const T* u, T* nu, hipStream_t s);
template <typename T>
hipError_t launch3_pc_diag(const Geo& g, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea,
                           hipStream_t s);
template <typename T>
hipError_t launch3_pc_sweep(const Geo& g, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                            const EpsArgs& ea, hipStream_t s);

// ---- vector kernels (vec.hip) ----
int red_blocks(long long n);
template <typename T>
hipError_t launch_norm2_partial(const T* x, long long n, double* partials, int nblk, hipStream_t s);
// out[k] = sum of partials[b * stride + k] over b < nblk, k < cnt (fixed order)
hipError_t launch_reduce_partials(const double* partials, int nblk, int stride, int cnt, double* out,
                                  int accumulate, hipStream_t s);
template <typename T>
hipError_t launch_multidot(const T* V, long long n, int nv, const T* w, double* partials, int nblk,
                           hipStream_t s);
// w -= sum_i h[i] V_i ; then partial dots of V_i with the new w (dots != 0) or partial ||w||^2
template <typename T>
hipError_t launch_update_dot(const T* V, long long n, int nv, const double* h, T* w, double* partials,
                             int nblk, int mode, hipStream_t s);
template <typename T>
hipError_t launch_scale(T* x, long long n, const double* inv_scale_dev, hipStream_t s);  // x /= *dev
template <typename T>
hipError_t launch_axpy_basis(T* x, const T* Z, long long n, int k, const double* y, hipStream_t s);
template <typename Td, typename Ts>
hipError_t launch_cast(Td* d, const Ts* s_, long long n, double alpha, hipStream_t s);   // d = alpha*s
template <typename Ts>
hipError_t launch_add_to64(double* u, const Ts* d, long long n, hipStream_t s);          // u += d
template <typename T>
hipError_t launch_axpby(T* y, const T* x, long long n, double a, double b, hipStream_t s); // y = a x + b y
template <typename T>
hipError_t launch_lincomb(T* out, const T* x, const T* y, long long n, double a, double b,
                          hipStream_t s);                                                 // out = a x + b y
// small single-thread kernels on the device scalars
hipError_t launch_fd_eps(const double* unorm2, const double* vnorm2, double sqrt_eps_mach, double sqrt_n,
                         double* eps, hipStream_t s);
hipError_t launch_givens(const GivensArgs& a, const double* wnorm2, hipStream_t s);
int cgs_blocks(long long n);
template <typename T>
hipError_t launch_cgs(const T* V, long long n, int nv, const double* hin, T* w, double* partials,
                      double* hout, int mode, const GivensArgs& ga, hipStream_t s);
hipError_t launch_eps_finish(int nblk, const EpsArgs& ea, hipStream_t s);
template <typename T>
hipError_t launch_normalize_copy(T* v, long long n, const double* div, T* z, const EpsArgs& ea, hipStream_t s);
// One-reduction Arnoldi step (classical Gram-Schmidt whose second projection
// and normalization of each basis vector are delayed to the next iteration's
// single reduction).  DgArgs points at the device state the finishing kernel
// reads and updates; see vec.hip.
struct DgArgs {
    double* H = nullptr;        // rotated Hessenberg, row-major (m + 1) x m
    double* Hraw = nullptr;     // unrotated, each column divided by its direction's scale
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;
    double* h1 = nullptr;       // first-projection coefficients of the newest column
    double* rs = nullptr;       // r_c, the norm of basis vector c before normalization
    double* coef = nullptr;     // update coefficients: a[kMaxDots], e[kMaxDots], 1/r, c_w
    double* host = nullptr;     // pinned (r_j, |g_j|) for the host's test
    int m = 0;
};
// Reduction of iteration j (with_w) or of the closing step of a cycle (!with_w,
// basis vector j alone): the pass over V and the finishing block.
template <typename T>
hipError_t launch_dg_reduce(const T* V, long long n, int j, bool with_w, double* partials, const DgArgs& a,
                            hipStream_t s);
// Update pass of iteration j: rows j and j + 1 of V become q_j and q~_{j+1}.
template <typename T>
// sq (may be null): per-block partial sums of the squares of the new row q~_{j+1}
hipError_t launch_dg_update(T* V, long long n, int j, const double* coef, hipStream_t s, double* sq = nullptr);
constexpr int kDgMaxRows = 32;          // basis vectors the one-reduction step handles
hipError_t launch_backsolve(const double* H, const double* g, int k, int m, double* y, hipStream_t s);
hipError_t launch_set_start(const double* beta2, double* g, double* beta, int m, hipStream_t s);

}  // namespace jfnk
