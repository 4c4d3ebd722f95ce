// Vector kernels of the Krylov solver: FP64-accumulated dot products and norms
// with a fixed reduction order (deterministic across runs), Gram-Schmidt basis
// updates, casts and the FP64 Givens / back-substitution steps of GMRES
// (Saad and Schultz 1986).

#include "jfnk_internal.hpp"
#include "reduce.hpp"

namespace jfnk {

namespace {

constexpr int kBlock = 256;
constexpr int kGroup = 8;        // basis vectors per register group of a dot pass

// Sum over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Block-wide sum of one value per thread (256 threads = 4 wavefronts); the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm2_partial(const T* __restrict__ x, long long n,
                                                          double* __restrict__ partials) {
    __shared__ double red[4];
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double v = (double)x[i];
        acc += v * v;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partials, int nblk,
                                                            int stride, double* __restrict__ out,
                                                            int accumulate) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    const double s = sum_partials(partials, nblk, stride, k, red);
    if (threadIdx.x == 0) out[k] = accumulate ? out[k] + s : s;
}

// partials[b * kMaxDots + v] = partial dot of V_v with w, v < nv
template <typename T>
__global__ __launch_bounds__(kBlock) void k_multidot(const T* __restrict__ V, long long n, int nv,
                                                     const T* __restrict__ w, double* __restrict__ partials) {
    __shared__ double red[4];
    const long long stride = (long long)gridDim.x * kBlock;
    for (int g0 = 0; g0 < nv; g0 += kGroup) {
        double acc[kGroup];
#pragma unroll
        for (int v = 0; v < kGroup; ++v) acc[v] = 0.0;
        const int cnt = nv - g0 < kGroup ? nv - g0 : kGroup;
        for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
            const double wv = (double)w[i];
#pragma unroll
            for (int v = 0; v < kGroup; ++v)
                if (v < cnt) acc[v] += (double)V[(long long)(g0 + v) * n + i] * wv;
        }
#pragma unroll
        for (int v = 0; v < kGroup; ++v) {
            if (v < cnt) {
                const double s = block_sum(acc[v], red);
                if (threadIdx.x == 0) partials[(long long)blockIdx.x * kMaxDots + g0 + v] = s;
            }
        }
    }
}

// w -= sum_v h[v] V_v; mode 1: also partial ||w||^2 into partials[b]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(const T* __restrict__ V, long long n, int nv,
                                                   const double* __restrict__ h, T* __restrict__ w,
                                                   double* __restrict__ partials, int mode) {
    __shared__ double red[4];
    __shared__ double hs[kMaxDots];
    for (int v = threadIdx.x; v < nv; v += kBlock) hs[v] = h[v];
    __syncthreads();
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double s = (double)w[i];
        for (int v = 0; v < nv; ++v) s -= hs[v] * (double)V[(long long)v * n + i];
        const T o = (T)s;
        w[i] = o;
        acc += (double)o * (double)o;
    }
    if (mode == 1) {
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_div(T* __restrict__ x, long long n,
                                                      const double* __restrict__ d) {
    const double den = *d;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        x[i] = (T)((double)x[i] / den);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_basis(T* __restrict__ x, const T* __restrict__ Z, long long n,
                                                       int k, const double* __restrict__ y) {
    __shared__ double ys[kMaxDots];
    for (int v = threadIdx.x; v < k; v += kBlock) ys[v] = y[v];
    __syncthreads();
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double s = (double)x[i];
        for (int v = 0; v < k; ++v) s += ys[v] * (double)Z[(long long)v * n + i];
        x[i] = (T)s;
    }
}

template <typename Td, typename Ts>
__global__ __launch_bounds__(kBlock) void k_cast(Td* __restrict__ d, const Ts* __restrict__ s, long long n,
                                                 double alpha) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        d[i] = (Td)(alpha * (double)s[i]);
}

template <typename Ts>
__global__ __launch_bounds__(kBlock) void k_add_to64(double* __restrict__ u, const Ts* __restrict__ d,
                                                     long long n) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        u[i] = u[i] + (double)d[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby(T* __restrict__ y, const T* __restrict__ x, long long n,
                                                  double a, double b) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        y[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_lincomb(T* __restrict__ o, const T* __restrict__ x,
                                                    const T* __restrict__ y, long long n, double a, double b) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        o[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}

// eps = sqrt(eps_mach) max(||u||, sqrt(N)) / ||v||   (0 when v = 0)
__global__ void k_fd_eps(const double* unorm2, const double* vnorm2, double sqrt_eps, double sqrt_n,
                         double* eps) {
    const double nv = sqrt(*vnorm2);
    const double nu = sqrt(*unorm2);
    *eps = nv > 0.0 ? sqrt_eps * (nu > sqrt_n ? nu : sqrt_n) / nv : 0.0;
}

// Column j of the Hessenberg: h1 + h2 above the diagonal, ||w|| below; apply the
// previous rotations, form the new one, update g and the residual estimate.
// Hraw (row-major (m+1) x m) keeps the unrotated column.
__device__ void givens_column(const GivensArgs& a, double wnorm2) {
    const int j = a.j, m = a.m;
    double* H = a.H;
    for (int i = 0; i <= j; ++i) {
        const double h = a.h1[i] + a.h2[i];
        H[i * m + j] = h;
        a.Hraw[i * m + j] = h;
    }
    const double nw = sqrt(wnorm2);
    H[(j + 1) * m + j] = nw;
    a.Hraw[(j + 1) * m + j] = nw;
    *a.wnorm = nw;
    for (int i = 0; i < j; ++i) {
        const double x = H[i * m + j], y = H[(i + 1) * m + j];
        H[i * m + j] = a.cs[i] * x + a.sn[i] * y;
        H[(i + 1) * m + j] = -a.sn[i] * x + a.cs[i] * y;
    }
    const double x = H[j * m + j], y = H[(j + 1) * m + j];
    const double r = hypot(x, y);
    double c = 1.0, sn = 0.0;
    if (r > 0.0) {
        c = x / r;
        sn = y / r;
    }
    a.cs[j] = c;
    a.sn[j] = sn;
    H[j * m + j] = r;
    H[(j + 1) * m + j] = 0.0;
    a.g[j + 1] = -sn * a.g[j];
    a.g[j] = c * a.g[j];
    *a.res_est = fabs(a.g[j + 1]);
    if (a.host) {                       // mirror for the host's convergence test
        a.host[0] = nw;
        a.host[1] = *a.res_est;
    }
}

__global__ void k_givens(GivensArgs a, const double* wnorm2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    givens_column(a, *wnorm2);
}

// Back substitution of the k x k upper triangle of H (row-major, row stride m)
// by columns: y_i = s_i / H_ii, then every row above subtracts H_li y_i.  One
// wavefront, H and g staged in LDS (k <= kMaxDots).
__global__ __launch_bounds__(64) void k_backsolve(const double* H, const double* g, int k, int m, double* y) {
    __shared__ double sH[kMaxDots][kMaxDots + 1];
    __shared__ double sy[kMaxDots];
    const int t = threadIdx.x;
    for (int idx = t; idx < k * k; idx += 64) {
        const int i = idx / k, l = idx - i * k;
        sH[i][l] = H[i * m + l];
    }
    double s = t < k ? g[t] : 0.0;
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        if (t == i) sy[i] = s / sH[i][i];
        __syncthreads();
        if (t < i) s -= sH[t][i] * sy[i];
    }
    __syncthreads();
    if (t < k) y[t] = sy[t];
}

__global__ void k_set_start(const double* beta2, double* g, double* beta, int m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double b = sqrt(*beta2);
    *beta = b;
    g[0] = b;
    for (int i = 1; i <= m; ++i) g[i] = 0.0;
}


// ---------------------------------------------------------------------------
// Fused classical Gram-Schmidt passes over the basis V_0..V_{nv-1}:
//   CGS_DOT       hout = V^T w
//   CGS_UPD_DOT   w <- w - V hin, hout = V^T w          (basis values reused from registers)
//   CGS_UPD_NORM  w <- w - V hin, ||w||^2, then the Givens step of column j
// Each block writes its partial sums; k_cgs_finish adds them in a fixed order.
// Up to 32 basis vectors the passes run in k_cgs_reg (basis in registers),
// beyond that in k_cgs (basis staged in LDS).
// ---------------------------------------------------------------------------
// k_cgs: chunks of kChunk consecutive elements; V_0..V_{nv-1} of the chunk are
// staged in LDS once; each thread updates its own element of w, then wavefront
// k forms the dots of basis vectors k, k+4, ... with the chunk of w (FP64
// accumulation).
constexpr int kChunk = 256;

template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_cgs(const T* __restrict__ V, long long n, int nv,
                                                const double* __restrict__ hin, T* __restrict__ w,
                                                double* __restrict__ partials, int mode) {
    __shared__ T sV[NV][kChunk];
    __shared__ T sW[kChunk];
    __shared__ double hs[NV];
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int v = tid; v < NV; v += kBlock) hs[v] = (mode != CGS_DOT && v < nv) ? hin[v] : 0.0;
    __syncthreads();
    constexpr int KPW = NV / 4;               // basis vectors per wavefront
    double acc[KPW];
#pragma unroll
    for (int k = 0; k < KPW; ++k) acc[k] = 0.0;
    double nacc = 0.0;
    const long long step = (long long)gridDim.x * kChunk;
    for (long long c0 = (long long)blockIdx.x * kChunk; c0 < n; c0 += step) {
        const long long i = c0 + tid;
        const bool ok = i < n;
        T wv = ok ? w[i] : T(0);
        double sacc = (double)wv;
        // groups of 8 independent loads in flight (row index clamped: always in bounds)
        for (int v0 = 0; v0 < nv; v0 += 8) {
            T x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int v = v0 + u < nv ? v0 + u : nv - 1;
                x[u] = ok ? V[(long long)v * n + i] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (v0 + u < nv) {
                    sV[v0 + u][tid] = x[u];
                    sacc -= hs[v0 + u] * (double)x[u];
                }
            }
        }
        if (mode != CGS_DOT) {
            wv = (T)sacc;
            if (ok) w[i] = wv;
        }
        if (mode == CGS_UPD_NORM) {
            nacc += (double)wv * (double)wv;
            continue;
        }
        sW[tid] = wv;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int v = wid + 4 * k;
            if (v < nv) {
                double a = 0.0;
#pragma unroll
                for (int t = lane; t < kChunk; t += 64) a += (double)sV[v][t] * (double)sW[t];
                acc[k] += a;
            }
        }
        __syncthreads();
    }
    if (mode == CGS_UPD_NORM) {
        const double t = block_sum256(nacc, red);
        if (tid == 0) partials[blockIdx.x] = t;
        return;
    }
#pragma unroll
    for (int k = 0; k < KPW; ++k) {
        const int v = wid + 4 * k;
        if (v < nv) {
            const double t = wave_sum64(acc[k]);
            if (lane == 0) partials[(long long)v * gridDim.x + blockIdx.x] = t;
        }
    }
}

// The same three passes with the basis held in registers instead of LDS: one
// element of w per thread and step, all NV basis loads of the element issued
// before any arithmetic (rows nv..NV-1 re-read row nv-1; their update
// coefficient is zero and their dots are never stored), the dots kept per
// thread in FP64 and reduced once per block.  No barrier inside the element
// loop, so the loads of one wavefront overlap the arithmetic of the others.
// A wavefront-uniform branch per row instead of the clamped re-read makes the
// compiler wait for each load before issuing the next.
template <typename T, int NV, int MODE>
__global__ __launch_bounds__(kBlock) void k_cgs_reg(const T* __restrict__ V, int n, int nv,
                                                    const double* __restrict__ hin, T* __restrict__ w,
                                                    double* __restrict__ partials) {
    constexpr bool kDots = MODE != CGS_UPD_NORM;
    constexpr bool kUpd = MODE != CGS_DOT;
    __shared__ double red[4][kDots ? NV : 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double h[NV];                              // update coefficients (wavefront-uniform)
#pragma unroll
    for (int v = 0; v < NV; ++v) h[v] = (kUpd && v < nv) ? hin[v] : 0.0;
    double acc[kDots ? NV : 1];
#pragma unroll
    for (int v = 0; v < (kDots ? NV : 1); ++v) acc[v] = 0.0;
    double nacc = 0.0;
    const int step = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + tid; i < n; i += step) {
        T wv = w[i];
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = V[(long long)(v < nv ? v : nv - 1) * n + i];
        // keep every load of the element ahead of its arithmetic (left alone, the
        // scheduler of the dot-only pass interleaves them and keeps ~5 in flight)
        __builtin_amdgcn_sched_barrier(0);
        if (kUpd) {
            double sacc = (double)wv;
#pragma unroll
            for (int v = 0; v < NV; ++v) sacc -= h[v] * (double)x[v];
            wv = (T)sacc;
            w[i] = wv;
        }
        if (kDots) {
            const double wd = (double)wv;
#pragma unroll
            for (int v = 0; v < (kDots ? NV : 1); ++v) acc[v] += (double)x[v] * wd;
        } else {
            nacc += (double)wv * (double)wv;
        }
    }
    if (!kDots) {
        const double t = block_sum256(nacc, &red[0][0]);
        if (tid == 0) partials[blockIdx.x] = t;
        return;
    }
    constexpr int kSpan = 64 / NV;             // lanes sharing one value after the scatter
    const double t = wave_sum_scatter<kDots ? NV : 1>(acc, lane);
    if (lane % kSpan == 0) red[wid][lane / kSpan] = t;
    __syncthreads();
    if (tid < nv)
        partials[(long long)tid * gridDim.x + blockIdx.x] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// Block v: hout[v] = sum of the pass partials (fixed order).  The last pass has
// a single value (||w||^2) and its block also takes the Givens step of column j.
__global__ __launch_bounds__(kBlock) void k_cgs_finish(const double* __restrict__ partials, int nblk,
                                                       double* __restrict__ hout, int mode, GivensArgs ga) {
    __shared__ double red[4];
    __shared__ double col[kMaxDots + 1], scs[kMaxDots], ssn[kMaxDots];
    const int v = blockIdx.x;
    const double t = sum_partials(partials + (long long)v * nblk, nblk, 1, 0, red);   // layout [v][block]
    if (threadIdx.x == 0) hout[v] = t;
    if (mode != CGS_UPD_NORM) return;
    // Givens step of column j: stage the column and the previous rotations in LDS
    const int j = ga.j, m = ga.m;
    for (int i = threadIdx.x; i <= j; i += kBlock) {
        col[i] = ga.h1[i] + ga.h2[i];
        ga.Hraw[i * m + j] = col[i];
        if (i < j) {
            scs[i] = ga.cs[i];
            ssn[i] = ga.sn[i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nw = sqrt(t);
        ga.Hraw[(j + 1) * m + j] = nw;
        *ga.wnorm = nw;
        col[j + 1] = nw;
        for (int i = 0; i < j; ++i) {
            const double x = col[i], y = col[i + 1];
            col[i] = scs[i] * x + ssn[i] * y;
            col[i + 1] = -ssn[i] * x + scs[i] * y;
        }
        const double x = col[j], y = col[j + 1];
        const double r = hypot(x, y);
        double c = 1.0, sn = 0.0;
        if (r > 0.0) {
            c = x / r;
            sn = y / r;
        }
        ga.cs[j] = c;
        ga.sn[j] = sn;
        col[j] = r;
        col[j + 1] = 0.0;
        const double gj = ga.g[j];
        ga.g[j + 1] = -sn * gj;
        ga.g[j] = c * gj;
        *ga.res_est = fabs(sn * gj);
        if (ga.host) {                   // pinned host mirror for the convergence test
            ga.host[0] = nw;
            ga.host[1] = fabs(sn * gj);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += kBlock) ga.H[i * m + j] = col[i];
}

// ---------------------------------------------------------------------------
// One-reduction Arnoldi step: classical Gram-Schmidt whose second projection
// and normalization of each basis vector are delayed to the next iteration's
// single reduction (the low-synchronization Gram-Schmidt of Swirydowicz et al.
// 2021 and Bielich et al. 2022).  At iteration j, row j of V holds q~_j (basis
// vector j after one projection, not normalized) and row j + 1 holds w = A z_j,
// z_j the preconditioned q~_j.  One pass forms per block
//     s_v = V_v . q~_j,  y_v = V_v . w  (v < j),  alpha = q~_j . q~_j,  beta = q~_j . w;
// one block adds them up and forms
//     r_j = sqrt(alpha - s.s)          norm of q~_j projected once more,
//     column j-1 = its first projection + s, subdiagonal r_j (final: Givens step),
//     h_j = (y, (beta - s.y) / r_j)    the first projection of w on q_0 .. q_j;
// a second pass overwrites row j with q_j = (q~_j - V_{<j} s) / r_j and row
// j + 1 with q~_{j+1} = (w - V_{<j} y - q_j h_jj) / r_j.  Without w (closing a
// cycle) only s and alpha are formed and column j-1 is finished.  z_j carries
// the scale r_j of q~_j; the Hessenberg columns keep it (the Arnoldi relation
// A Z = V H holds for the stored Z): column j-1 = (its first projection
// + r_{j-1} s, r_{j-1} r_j), the returned raw columns are divided by it.  The
// division of q~_{j+1} by r_j keeps the scales from compounding over a cycle
// (they would grow like the product of the subdiagonal, past the FP32 range
// of the products inside the Jacobian-vector step).
// ---------------------------------------------------------------------------
constexpr int kDgBlocks = 256;          // blocks of the reduction pass
constexpr int kDgSlots = 2 * kDgMaxRows + 2;
enum { DG_S = 0, DG_Y = kDgMaxRows, DG_ALPHA = 2 * kDgMaxRows, DG_BETA = 2 * kDgMaxRows + 1 };
constexpr int kDgCoefW = kMaxDots;      // coef layout: a[0..), e[kDgCoefW..), 1/r, c_w at 2 kDgCoefW

template <typename T, int NV, bool W, int NT>
__global__ __launch_bounds__(NT) void k_dg_dot(const T* __restrict__ V, int n, int j, double* __restrict__ partials) {
    constexpr int NA = W ? 2 * NV : NV;       // row dots per thread: s, then y
    constexpr int NW = NT / 64;
    __shared__ double red[NW][NA + 2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const T* q = V + (long long)j * n;
    const T* w = V + (long long)(j + 1) * n;
    const int last = j > 0 ? j - 1 : 0;        // rows past j - 1 re-read row j - 1 (row 0 when j = 0)
    double acc[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) acc[v] = 0.0;
    double aa = 0.0, ab = 0.0;
    const int step = gridDim.x * NT;
    for (int i = blockIdx.x * NT + tid; i < n; i += step) {
        const T qv = q[i];
        const T wv = W ? w[i] : T(0);
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = V[(long long)(v < j ? v : last) * n + i];
        __builtin_amdgcn_sched_barrier(0);    // all loads of the element ahead of its arithmetic
        const double qd = (double)qv, wd = (double)wv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            acc[v] += (double)x[v] * qd;
            if (W) acc[NV + v] += (double)x[v] * wd;
        }
        aa += qd * qd;
        if (W) ab += qd * wd;
    }
    constexpr int kSpan = 64 / NA;
    const double t = wave_sum_scatter<NA>(acc, lane);
    if (lane % kSpan == 0) red[wid][lane / kSpan] = t;
    const double ta = wave_sum64(aa);
    const double tb = W ? wave_sum64(ab) : 0.0;
    if (lane == 0) {
        red[wid][NA] = ta;
        red[wid][NA + 1] = tb;
    }
    __syncthreads();
    for (int o = tid; o < NA + 2; o += NT) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) sum += red[k][o];
        int slot = -1;
        if (o < NV) {
            if (o < j) slot = DG_S + o;
        } else if (o < NA) {
            if (o - NV < j) slot = DG_Y + (o - NV);
        } else if (o == NA) {
            slot = DG_ALPHA;
        } else if (W) {
            slot = DG_BETA;
        }
        if (slot >= 0) partials[(long long)slot * gridDim.x + blockIdx.x] = sum;
    }
}

// One block of 1024 threads: the sums of the pass; then wavefront 0, one lane
// per basis vector, the closed column j-1 and the coefficients of the update
// pass; then thread 0 the Givens step of column j-1 (FP64 throughout).
__global__ __launch_bounds__(1024) void k_dg_finish(const double* __restrict__ partials, int nb, int j, int with_w,
                                                    DgArgs a) {
    __shared__ double sums[kDgSlots];
    __shared__ double hp[kMaxDots + 1], scs[kMaxDots], ssn[kMaxDots], pre[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int o = wid; o < kDgSlots; o += 16) {          // one output per wavefront at a time
        const bool need = o < DG_Y ? o < j : o < DG_ALPHA ? (with_w && o - DG_Y < j) : (o == DG_ALPHA || with_w);
        if (!need) continue;
        double acc = 0.0;
        for (int b0 = lane; b0 < nb; b0 += 8 * 64) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u * 64;
                x[u] = b < nb ? partials[(long long)o * nb + b] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += x[u];
        }
        acc = wave_sum64(acc);
        if (lane == 0) sums[o] = acc;
    }
    for (int i = tid; i < j; i += 1024) {
        hp[i] = a.h1[i];                                 // first projection of column j-1
        scs[i] = a.cs[i];
        ssn[i] = a.sn[i];
    }
    if (tid == 1023 && j > 0) {                          // the scale of z_{j-1} and g_{j-1}
        pre[0] = a.rs[j - 1];
        pre[1] = a.g[j - 1];
    }
    __syncthreads();
    const int m = a.m;
    // wavefront 0, one lane per basis vector (j < 32): s.s and s.y, the closed
    // column j-1 before its rotations, and the update coefficients
    if (wid == 0) {
        const double sv = lane < j ? sums[DG_S + lane] : 0.0;
        const double yv = (with_w && lane < j) ? sums[DG_Y + lane] : 0.0;
        double ss = sv * sv, sy = sv * yv;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {               // butterfly: the same sums in every lane
            ss += __shfl_xor(ss, o, 64);
            sy += __shfl_xor(sy, o, 64);
        }
        const double r2 = sums[DG_ALPHA] - ss;
        // a NaN (a non-finite Krylov vector) stays NaN for the host's test
        const double r = r2 > 0.0 ? sqrt(r2) : (r2 != r2 ? r2 : 0.0);
        if (j > 0) {
            const double sc = pre[0];
            const double inv_sc = sc > 0.0 ? 1.0 / sc : 0.0;
            double h = 0.0;
            if (lane < j) h = hp[lane] + sc * sv;
            else if (lane == j) h = sc * r;
            if (lane <= j) {
                hp[lane] = h;
                a.Hraw[lane * m + (j - 1)] = h * inv_sc;
            }
        }
        if (with_w) {
            const double inv_r = r > 0.0 ? 1.0 / r : 0.0;
            const double hjj = (sums[DG_BETA] - sy) * inv_r;
            const double cw = hjj * inv_r;
            if (lane < j) {
                a.coef[lane] = sv;
                a.coef[kDgCoefW + lane] = yv - cw * sv;
            }
            if (lane == 0) {
                a.coef[2 * kDgCoefW] = inv_r;
                a.coef[2 * kDgCoefW + 1] = cw;
                pre[2] = hjj;
            }
        }
        if (lane == 0) pre[3] = r;
    }
    __syncthreads();
    if (with_w && tid < j) a.h1[tid] = sums[DG_Y + tid];   // after every read of the old h1
    if (tid != 0) return;
    const double r = pre[3];
    double res = 0.0;
    if (j == 0) {
        a.g[0] = r;                                      // the start vector is r q_0
    } else {
        // Givens rotations of column c = j-1, the rotated value carried in a register
        const int c = j - 1;
        double y = hp[0];
        for (int i = 0; i < c; ++i) {
            const double z = hp[i + 1];
            a.H[i * m + c] = scs[i] * y + ssn[i] * z;
            y = -ssn[i] * y + scs[i] * z;
        }
        const double z = hp[c + 1];
        const double rr = hypot(y, z);
        double cc = 1.0, sn = 0.0;
        if (rr > 0.0) {
            cc = y / rr;
            sn = z / rr;
        }
        a.cs[c] = cc;
        a.sn[c] = sn;
        a.H[c * m + c] = rr;
        a.H[(c + 1) * m + c] = 0.0;
        const double gc = pre[1];
        a.g[c + 1] = -sn * gc;
        a.g[c] = cc * gc;
        res = fabs(sn * gc);
    }
    a.rs[j] = r;
    if (with_w) a.h1[j] = pre[2];
    if (a.host) {
        a.host[0] = r;
        a.host[1] = res;
    }
}

// q_j = (q~_j - sum_v a_v V_v) / r_j over row j, and over row j + 1
// (w - c_w q~_j - sum_v e_v V_v) / r_j  (e_v = y_v - c_w a_v, c_w = h_jj / r_j).
//
// With sq set, each block also leaves the partial sum of the new row's squares
// in sq[block]: the learned preconditioner, which acts on that row next, takes
// its input scale from them instead of another pass over the row.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename T, int NV, bool NT>
__global__ __launch_bounds__(kBlock) void k_dg_update(T* V, int n, int j, const double* __restrict__ coef,
                                                      double* __restrict__ sq) {
    __shared__ double red[4];
    T* q = V + (long long)j * n;
    T* w = V + (long long)(j + 1) * n;
    const int last = j > 0 ? j - 1 : 0;
    double ca[NV], ce[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ca[v] = v < j ? coef[v] : 0.0;
        ce[v] = v < j ? coef[kDgCoefW + v] : 0.0;
    }
    const double inv_r = coef[2 * kDgCoefW], cw = coef[2 * kDgCoefW + 1];
    const int step = gridDim.x * kBlock;
    double acc = 0.0;
    // NT: every value is touched once here, so on a basis far beyond the
    // Infinity Cache the loads and stores take the streaming (non-temporal)
    // path, 4% more bandwidth than cached accesses at 5 x 8.4 M points.  A
    // basis the cache holds keeps cached accesses (streaming costs 6% there).
    // The reduction pass keeps cached loads (3% slower when streamed): this
    // pass reads its rows again right after it.
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const T qv = ld_stream<NT>(q + i), wv = ld_stream<NT>(w + i);
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = ld_stream<NT>(V + (long long)(v < j ? v : last) * n + i);
        __builtin_amdgcn_sched_barrier(0);
        double sqv = (double)qv, sw = (double)wv - cw * (double)qv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sqv -= ca[v] * (double)x[v];
            sw -= ce[v] * (double)x[v];
        }
        st_stream<NT>((T)(sqv * inv_r), q + i);
        const T wn = (T)(sw * inv_r);
        st_stream<NT>(wn, w + i);
        acc += (double)wn * (double)wn;
    }
    if (sq) {
        const double t = block_sum256(acc, red);
        if (threadIdx.x == 0) sq[blockIdx.x] = t;
    }
}

// x += sum_v y_v Z_v for k <= NV basis rows, every row's load of an element
// issued before the sums (the loop form above keeps one load in flight); rows
// past k - 1 re-read row k - 1 with a zero coefficient.  The sums run in the
// loop form's order.  NT: streaming loads of Z as in the Arnoldi update pass.
template <typename T, int NV, bool NT>
__global__ __launch_bounds__(kBlock) void k_axpy_basis_reg(T* __restrict__ x, const T* __restrict__ Z, int n, int k,
                                                           const double* __restrict__ y) {
    double c[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = v < k ? y[v] : 0.0;
    const int step = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        T z[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = ld_stream<NT>(Z + (long long)(v < k ? v : k - 1) * n + i);
        __builtin_amdgcn_sched_barrier(0);
        double acc = (double)x[i];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc += c[v] * (double)z[v];
        x[i] = (T)acc;
    }
}

__global__ __launch_bounds__(kBlock) void k_eps_finish(int nblk, EpsArgs ea) {
    __shared__ double red[4];
    const double t = sum_partials(ea.partials, nblk, 1, 0, red);
    if (threadIdx.x == 0) finish_eps(ea, t);
}

// v <- v / *div (if div), z = v; partial ||z||^2 for the FD step
template <typename T>
__global__ __launch_bounds__(kBlock) void k_normalize_copy(T* __restrict__ v, long long n,
                                                           const double* __restrict__ div, T* __restrict__ z,
                                                           EpsArgs ea) {
    __shared__ double red[4];
    const double d = div ? *div : 1.0;
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        T o = v[i];
        if (div) {
            o = (T)((double)o / d);
            v[i] = o;
        }
        z[i] = o;
        acc += (double)o * (double)o;
    }
    if (ea.partials) partial_eps(ea, acc, red);
}

int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int red_blocks(long long n) {
    long long b = (n + 4LL * kBlock - 1) / (4LL * kBlock);
    if (b > kMaxPartials) b = kMaxPartials;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename T>
hipError_t launch_norm2_partial(const T* x, long long n, double* partials, int nblk, hipStream_t s) {
    hipLaunchKernelGGL((k_norm2_partial<T>), dim3(nblk), dim3(kBlock), 0, s, x, n, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int nblk, int stride, int cnt, double* out,
                                  int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(cnt), dim3(kBlock), 0, s, partials, nblk, stride, out, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_multidot(const T* V, long long n, int nv, const T* w, double* partials, int nblk,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_multidot<T>), dim3(nblk), dim3(kBlock), 0, s, V, n, nv, w, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_dot(const T* V, long long n, int nv, const double* h, T* w, double* partials,
                             int nblk, int mode, hipStream_t s) {
    hipLaunchKernelGGL((k_update<T>), dim3(nblk), dim3(kBlock), 0, s, V, n, nv, h, w, partials, mode);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(T* x, long long n, const double* d, hipStream_t s) {
    hipLaunchKernelGGL((k_scale_div<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, n, d);
    return hipGetLastError();
}

template <typename T, int NV, bool NT>
hipError_t launch_axpy_basis_nv(T* x, const T* Z, int n, int k, const double* y, hipStream_t s) {
    hipLaunchKernelGGL((k_axpy_basis_reg<T, NV, NT>), dim3(cgs_blocks(n)), dim3(kBlock), 0, s, x, Z, n, k, y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_basis(T* x, const T* Z, long long n, int k, const double* y, hipStream_t s) {
    if (k < 1 || k > 32 || n >= (1LL << 30)) {
        hipLaunchKernelGGL((k_axpy_basis<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, x, Z, n, k, y);
        return hipGetLastError();
    }
    const int ni = (int)n;
    if (n * (long long)sizeof(T) >= (32LL << 20))
        return k <= 8 ? launch_axpy_basis_nv<T, 8, true>(x, Z, ni, k, y, s)
             : k <= 16 ? launch_axpy_basis_nv<T, 16, true>(x, Z, ni, k, y, s)
                       : launch_axpy_basis_nv<T, 32, true>(x, Z, ni, k, y, s);
    return k <= 8 ? launch_axpy_basis_nv<T, 8, false>(x, Z, ni, k, y, s)
         : k <= 16 ? launch_axpy_basis_nv<T, 16, false>(x, Z, ni, k, y, s)
                   : launch_axpy_basis_nv<T, 32, false>(x, Z, ni, k, y, s);
}

template <typename Td, typename Ts>
hipError_t launch_cast(Td* d, const Ts* s_, long long n, double alpha, hipStream_t s) {
    hipLaunchKernelGGL((k_cast<Td, Ts>), dim3(grid_for(n)), dim3(kBlock), 0, s, d, s_, n, alpha);
    return hipGetLastError();
}

template <typename Ts>
hipError_t launch_add_to64(double* u, const Ts* d, long long n, hipStream_t s) {
    hipLaunchKernelGGL((k_add_to64<Ts>), dim3(grid_for(n)), dim3(kBlock), 0, s, u, d, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axpby(T* y, const T* x, long long n, double a, double b, hipStream_t s) {
    hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, y, x, n, a, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lincomb(T* out, const T* x, const T* y, long long n, double a, double b, hipStream_t s) {
    hipLaunchKernelGGL((k_lincomb<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, out, x, y, n, a, b);
    return hipGetLastError();
}

hipError_t launch_fd_eps(const double* unorm2, const double* vnorm2, double sqrt_eps_mach, double sqrt_n,
                         double* eps, hipStream_t s) {
    hipLaunchKernelGGL(k_fd_eps, dim3(1), dim3(1), 0, s, unorm2, vnorm2, sqrt_eps_mach, sqrt_n, eps);
    return hipGetLastError();
}

hipError_t launch_givens(const GivensArgs& a, const double* wnorm2, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, s, a, wnorm2);
    return hipGetLastError();
}

int cgs_blocks(long long n) {
    long long b = (n + 8LL * kChunk - 1) / (8LL * kChunk);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename T, int NV, int MODE>
hipError_t launch_cgs_reg_mode(const T* V, int n, int nv, const double* hin, T* w, double* partials, int nb,
                               hipStream_t s) {
    hipLaunchKernelGGL((k_cgs_reg<T, NV, MODE>), dim3(nb), dim3(kBlock), 0, s, V, n, nv, hin, w, partials);
    return hipGetLastError();
}

template <typename T, int NV>
hipError_t launch_cgs_reg_nv(const T* V, int n, int nv, const double* hin, T* w, double* partials, int mode,
                             int nb, hipStream_t s) {
    if (mode == CGS_DOT) return launch_cgs_reg_mode<T, NV, CGS_DOT>(V, n, nv, hin, w, partials, nb, s);
    if (mode == CGS_UPD_DOT) return launch_cgs_reg_mode<T, NV, CGS_UPD_DOT>(V, n, nv, hin, w, partials, nb, s);
    return launch_cgs_reg_mode<T, NV, CGS_UPD_NORM>(V, n, nv, hin, w, partials, nb, s);
}

template <typename T>
hipError_t launch_cgs_reg(const T* V, int n, int nv, const double* hin, T* w, double* partials, int mode, int nb,
                          hipStream_t s) {
    if (nv <= 8) return launch_cgs_reg_nv<T, 8>(V, n, nv, hin, w, partials, mode, nb, s);
    if (nv <= 16) return launch_cgs_reg_nv<T, 16>(V, n, nv, hin, w, partials, mode, nb, s);
    return launch_cgs_reg_nv<T, 32>(V, n, nv, hin, w, partials, mode, nb, s);
}

template <typename T>
hipError_t launch_cgs(const T* V, long long n, int nv, const double* hin, T* w, double* partials,
                      double* hout, int mode, const GivensArgs& ga, hipStream_t s) {
    const int nb = cgs_blocks(n);
    if (nv <= 32 && n < (1LL << 30)) {   // int element index with room for the grid stride
        const hipError_t e = launch_cgs_reg<T>(V, (int)n, nv, hin, w, partials, mode, nb, s);
        if (e != hipSuccess) return e;
    } else if (nv <= 8)
        hipLaunchKernelGGL((k_cgs<T, 8>), dim3(nb), dim3(kBlock), 0, s, V, n, nv, hin, w, partials, mode);
    else if (nv <= 16)
        hipLaunchKernelGGL((k_cgs<T, 16>), dim3(nb), dim3(kBlock), 0, s, V, n, nv, hin, w, partials, mode);
    else if (nv <= 32)
        hipLaunchKernelGGL((k_cgs<T, 32>), dim3(nb), dim3(kBlock), 0, s, V, n, nv, hin, w, partials, mode);
    else
        hipLaunchKernelGGL((k_cgs<T, 64>), dim3(nb), dim3(kBlock), 0, s, V, n, nv, hin, w, partials, mode);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nacc = mode == CGS_UPD_NORM ? 1 : nv;
    hipLaunchKernelGGL(k_cgs_finish, dim3(nacc), dim3(kBlock), 0, s, partials, nb, hout, mode, ga);
    return hipGetLastError();
}

template <typename T, int NV, bool W, int NT>
hipError_t launch_dg_dot_nv(const T* V, int n, int j, double* partials, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_dg_dot<T, NV, W, NT>), dim3(nb), dim3(NT), 0, s, V, n, j, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_reduce(const T* V, long long n, int j, bool with_w, double* partials, const DgArgs& a,
                            hipStream_t s) {
    if (j < 0 || j >= kDgMaxRows || n < 1 || n >= (1LL << 30)) return hipErrorInvalidValue;
    // threads per block: 1024 while the dots fit 128 registers; 512 for 32 rows
    // with w, or 32 FP64 rows
    const int nt = (j > 16 && (with_w || sizeof(T) == 8)) ? 512 : 1024;
    long long nb = (n + nt - 1) / nt;
    if (nb > kDgBlocks) nb = kDgBlocks;
    const int ni = (int)n, b = (int)nb;
    hipError_t e;
    if (with_w) {
        e = j <= 8 ? launch_dg_dot_nv<T, 8, true, 1024>(V, ni, j, partials, b, s)
          : j <= 16 ? launch_dg_dot_nv<T, 16, true, 1024>(V, ni, j, partials, b, s)
                    : launch_dg_dot_nv<T, 32, true, 512>(V, ni, j, partials, b, s);
    } else {
        constexpr int kNt32 = sizeof(T) == 8 ? 512 : 1024;
        e = j <= 8 ? launch_dg_dot_nv<T, 8, false, 1024>(V, ni, j, partials, b, s)
          : j <= 16 ? launch_dg_dot_nv<T, 16, false, 1024>(V, ni, j, partials, b, s)
                    : launch_dg_dot_nv<T, 32, false, kNt32>(V, ni, j, partials, b, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dg_finish, dim3(1), dim3(1024), 0, s, (const double*)partials, b, j, with_w ? 1 : 0, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_update(T* V, long long n, int j, const double* coef, hipStream_t s, double* sq) {
    if (j < 0 || j >= kDgMaxRows || n < 1 || n >= (1LL << 30)) return hipErrorInvalidValue;
    const int nb = cgs_blocks(n), ni = (int)n;
    // streaming accesses once 8 rows exceed the 256 MB Infinity Cache
    if (n * (long long)sizeof(T) >= (32LL << 20)) {
        if (j <= 8)
            hipLaunchKernelGGL((k_dg_update<T, 8, true>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
        else if (j <= 16)
            hipLaunchKernelGGL((k_dg_update<T, 16, true>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
        else
            hipLaunchKernelGGL((k_dg_update<T, 32, true>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
    } else {
        if (j <= 8)
            hipLaunchKernelGGL((k_dg_update<T, 8, false>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
        else if (j <= 16)
            hipLaunchKernelGGL((k_dg_update<T, 16, false>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
        else
            hipLaunchKernelGGL((k_dg_update<T, 32, false>), dim3(nb), dim3(kBlock), 0, s, V, ni, j, coef, sq);
    }
    return hipGetLastError();
}

hipError_t launch_eps_finish(int nblk, const EpsArgs& ea, hipStream_t s) {
    hipLaunchKernelGGL(k_eps_finish, dim3(1), dim3(kBlock), 0, s, nblk, ea);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_normalize_copy(T* v, long long n, const double* div, T* z, const EpsArgs& ea, hipStream_t s) {
    hipLaunchKernelGGL((k_normalize_copy<T>), dim3(cgs_blocks(n)), dim3(kBlock), 0, s, v, n, div, z, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    return launch_eps_finish(cgs_blocks(n), ea, s);
}

hipError_t launch_backsolve(const double* H, const double* g, int k, int m, double* y, hipStream_t s) {
    if (k < 1 || k > kMaxDots) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, H, g, k, m, y);
    return hipGetLastError();
}

hipError_t launch_set_start(const double* beta2, double* g, double* beta, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_set_start, dim3(1), dim3(1), 0, s, beta2, g, beta, m);
    return hipGetLastError();
}

#define JFNK_VINST(T)                                                                                          \
    template hipError_t launch_norm2_partial<T>(const T*, long long, double*, int, hipStream_t);               \
    template hipError_t launch_multidot<T>(const T*, long long, int, const T*, double*, int, hipStream_t);      \
    template hipError_t launch_update_dot<T>(const T*, long long, int, const double*, T*, double*, int, int,   \
                                             hipStream_t);                                                     \
    template hipError_t launch_scale<T>(T*, long long, const double*, hipStream_t);                            \
    template hipError_t launch_axpy_basis<T>(T*, const T*, long long, int, const double*, hipStream_t);        \
    template hipError_t launch_add_to64<T>(double*, const T*, long long, hipStream_t);                         \
    template hipError_t launch_axpby<T>(T*, const T*, long long, double, double, hipStream_t);                 \
    template hipError_t launch_lincomb<T>(T*, const T*, const T*, long long, double, double, hipStream_t); \
    template hipError_t launch_cgs<T>(const T*, long long, int, const double*, T*, double*, double*, int,      \
                                      const GivensArgs&, hipStream_t);                                         \
    template hipError_t launch_normalize_copy<T>(T*, long long, const double*, T*, const EpsArgs&, hipStream_t); \
    template hipError_t launch_dg_reduce<T>(const T*, long long, int, bool, double*, const DgArgs&, hipStream_t); \
    template hipError_t launch_dg_update<T>(T*, long long, int, const double*, hipStream_t, double*);
JFNK_VINST(double)
JFNK_VINST(float)
#undef JFNK_VINST
template hipError_t launch_cast<float, double>(float*, const double*, long long, double, hipStream_t);
template hipError_t launch_cast<double, float>(double*, const float*, long long, double, hipStream_t);
template hipError_t launch_cast<double, double>(double*, const double*, long long, double, hipStream_t);
template hipError_t launch_cast<float, float>(float*, const float*, long long, double, hipStream_t);

}  // namespace jfnk
