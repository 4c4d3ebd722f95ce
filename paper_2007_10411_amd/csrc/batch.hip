// Batched ensemble of independent 2D problems of uneven sizes, solved together:
// every stage of the Newton-Krylov iteration is ONE launch over all instances.
// Work-lists (prefix sums per instance of stencil tiles, point blocks and
// vector chunks) map each workgroup to its instance by binary search; per
// instance geometry, Krylov scalars, Givens rotations and an "active" mask live
// in device arrays, so instances that have converged drop out of the launches
// while the others continue in lockstep.
//
// State vectors of the batch are the instances' vectors back to back (instance
// i at element offset voff[i], each in the single-problem layout).

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "stencil2d_impl.hpp"

using jfnk::Geo;

namespace jfnk {
namespace {

constexpr int kB = 256;
constexpr int kChunk = 2048;            // elements per vector chunk (8 per thread)
constexpr int M = kMaxDots;             // per-instance stride of Krylov scalars

// Device view of a batch.
struct BTab {
    int ninst;
    const Geo* geos;
    const long long* voff;      // [ninst + 1] element offsets of the instances
    const long long* poff;      // [ninst + 1] grid-point offsets
    const long long* noff;      // [ninst + 1] offsets of the ring-W extended grids
    const int* tile_off;        // [ninst + 1] stencil tiles (for the tile height in use)
    const int* tiles_x;         // [ninst] tiles per row
    const int* pblk_off;        // [ninst + 1] blocks of 256 grid points
    const int* eblk_off;        // [ninst + 1] blocks of 256 extended points
    const int* chunk_off;       // [ninst + 1] vector chunks
    const int* active;          // [ninst] 1 = participates (null: all)
};

__device__ __forceinline__ int find_inst(const int* off, int n, int b) {
    int lo = 0, hi = n;                    // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool inactive(const BTab& t, int i) { return t.active && !t.active[i]; }

// ---------------------------------------------------------------------------
// stencil stages
// ---------------------------------------------------------------------------
// W: stencil half-width of every instance (2 for p = 2, 4 for p = 3)
template <typename T, int TZ, int W>
__global__ __launch_bounds__(kB) void kb_apply_F(BTab t, const T* __restrict__ u, const T* __restrict__ f,
                                                 T* __restrict__ out, int what) {
    const int i = find_inst(t.tile_off, t.ninst, blockIdx.x);
    if (inactive(t, i)) return;
    const Geo g = t.geos[i];
    const int local = blockIdx.x - t.tile_off[i];
    const int tx = local % t.tiles_x[i], tz = local / t.tiles_x[i];
    const long long o = t.voff[i];
    s2d::apply_F_tile<T, 64, TZ, W>(g, tx * 64, tz * TZ, u + o, f ? f + o : nullptr, out + o, what);
}

// FP64 tiles stop at 8 rows (4 for W = 4) for LDS, as in the single-grid kernels
template <typename T, int TZ, int W>
__global__ __launch_bounds__(kB) void kb_jv(BTab t, const T* __restrict__ u, const T* __restrict__ v,
                                            const double* __restrict__ eps, T* __restrict__ out) {
    constexpr int TZC = sizeof(T) == 8 ? (W == 4 ? 4 : (TZ > 8 ? 8 : TZ)) : TZ;
    const int i = find_inst(t.tile_off, t.ninst, blockIdx.x);
    if (inactive(t, i)) return;
    const Geo g = t.geos[i];
    const int local = blockIdx.x - t.tile_off[i];
    const int tx = local % t.tiles_x[i], tz = local / t.tiles_x[i];
    const long long o = t.voff[i];
    s2d::jv_tile<T, 64, TZC, W>(g, tx * 64, tz * TZC, u + o, v + o, 0.0,
                                eps ? eps + (long long)i * S_STRIDE : nullptr, out + o);
}

template <typename T, int TZ, int W>
__global__ __launch_bounds__(kB) void kb_pc_sweep(BTab t, const T* __restrict__ u, const T* __restrict__ nu,
                                                  const T* __restrict__ r, const T* __restrict__ zin,
                                                  T* __restrict__ zout) {
    static_assert(sizeof(T) == 4 || W == 2 || TZ <= 8, "FP64 sweep tiles with W = 4 stop at 8 rows");
    const int i = find_inst(t.tile_off, t.ninst, blockIdx.x);
    if (inactive(t, i)) return;
    const Geo g = t.geos[i];
    const int local = blockIdx.x - t.tile_off[i];
    const int tx = local % t.tiles_x[i], tz = local / t.tiles_x[i];
    const long long o = t.voff[i];
    (void)s2d::pc_sweep_tile<T, 64, TZ, W>(g, tx * 64, tz * TZ, u + o, nu + t.noff[i], r + o, zin + o, zout + o);
}

template <typename T, int W>
__global__ __launch_bounds__(kB) void kb_frozen_nu(BTab t, const T* __restrict__ u, T* __restrict__ nu) {
    const int i = find_inst(t.eblk_off, t.ninst, blockIdx.x);
    if (inactive(t, i)) return;
    const Geo g = t.geos[i];
    const long long k = (long long)(blockIdx.x - t.eblk_off[i]) * kB + threadIdx.x;
    s2d::frozen_nu_point<T, W>(g, k, u + t.voff[i], nu + t.noff[i]);
}

// z = v / d after v = V_j / div[i] is written back into V_j
template <typename T, int W>
__global__ __launch_bounds__(kB) void kb_pc_diag(BTab t, const T* __restrict__ nu, T* __restrict__ vj,
                                                 const double* __restrict__ div, T* __restrict__ z) {
    const int i = find_inst(t.pblk_off, t.ninst, blockIdx.x);
    if (inactive(t, i)) return;
    const Geo g = t.geos[i];
    const long long k = (long long)(blockIdx.x - t.pblk_off[i]) * kB + threadIdx.x;
    if (k >= g.npts) return;
    const long long o = t.voff[i];
    (void)s2d::pc_diag_point<T, W>(g, k, nu + t.noff[i], vj + o, div ? div + (long long)i * S_STRIDE : nullptr,
                                z + o);
}

// ---------------------------------------------------------------------------
// vector stages over chunks; per-instance reductions
// ---------------------------------------------------------------------------
struct Chunk {
    int inst;
    long long b, e;    // element range of the chunk
};
__device__ __forceinline__ Chunk chunk_of(const BTab& t) {
    Chunk c;
    c.inst = find_inst(t.chunk_off, t.ninst, blockIdx.x);
    const long long s0 = t.voff[c.inst] + (long long)(blockIdx.x - t.chunk_off[c.inst]) * kChunk;
    c.b = s0;
    c.e = min(s0 + kChunk, t.voff[c.inst + 1]);
    return c;
}

// partials[chunk] = sum of x^2 over the chunk (per-instance sums by kb_finish)
template <typename T>
__global__ __launch_bounds__(kB) void kb_norm2(BTab t, const T* __restrict__ x, double* __restrict__ partials) {
    __shared__ double red[4];
    const Chunk c = chunk_of(t);
    double acc = 0.0;
    if (!inactive(t, c.inst))
        for (long long k = c.b + threadIdx.x; k < c.e; k += kB) {
            const double v = (double)x[k];
            acc += v * v;
        }
    const double s = block_sum256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// per instance i (block i): out[i * stride] = sum of partials over i's chunks;
// then an optional finishing step on the instance's scalars
enum { FIN_STORE = 0, FIN_BETA = 1, FIN_EPS = 2 };
__global__ __launch_bounds__(kB) void kb_finish(BTab t, const double* __restrict__ partials, double* out,
                                                int stride, int mode, double* scal, double sqrt_eps) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    if (inactive(t, i)) return;
    double acc = 0.0;
    for (int b = t.chunk_off[i] + threadIdx.x; b < t.chunk_off[i + 1]; b += kB) acc += partials[b];
    const double s = block_sum256(acc, red);
    if (threadIdx.x != 0) return;
    out[(long long)i * stride] = s;
    double* sc = scal + (long long)i * S_STRIDE;
    if (mode == FIN_BETA) {                 // start of a cycle: g = (beta, 0, ...)
        const double b = sqrt(s);
        sc[SB_BETA] = b;
    } else if (mode == FIN_EPS) {           // FD step for the direction whose norm was summed
        const double nv = sqrt(s);
        const double nu = sqrt(sc[SB_UNORM2]);
        const double sn = sc[SB_SQRTN];
        sc[SB_EPS] = nv > 0.0 ? sqrt_eps * (nu > sn ? nu : sn) / nv : 0.0;
    }
}

// Gram-Schmidt passes, one chunk per block, basis vectors j of all instances at
// V + j * ntot (modes as in the single-problem pass); basis staged in LDS, used
// beyond 32 basis vectors (kb_cgs_reg below up to 32)
template <typename T, int NV>
__global__ __launch_bounds__(kB) void kb_cgs(BTab t, const T* __restrict__ V, long long ntot, int nv,
                                             const double* __restrict__ hin, T* __restrict__ w,
                                             double* __restrict__ partials, int nchunks, int mode) {
    __shared__ T sV[NV][kB];
    __shared__ T sW[kB];
    __shared__ double hs[NV];
    __shared__ double red[4];
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int v = tid; v < NV; v += kB) hs[v] = (mode != CGS_DOT && v < nv) ? hin[(long long)c.inst * M + v] : 0.0;
    __syncthreads();
    constexpr int KPW = NV / 4;
    double acc[KPW];
#pragma unroll
    for (int k = 0; k < KPW; ++k) acc[k] = 0.0;
    double nacc = 0.0;
    for (long long c0 = c.b; c0 < c.e; c0 += kB) {
        const long long i = c0 + tid;
        const bool ok = i < c.e;
        T wv = ok ? w[i] : T(0);
        double sacc = (double)wv;
        for (int v0 = 0; v0 < nv; v0 += 8) {
            T x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int v = v0 + u < nv ? v0 + u : nv - 1;
                x[u] = ok ? V[(long long)v * ntot + i] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (v0 + u < nv) {
                    sV[v0 + u][tid] = x[u];
                    sacc -= hs[v0 + u] * (double)x[u];
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
                for (int q = lane; q < kB; q += 64) a += (double)sV[v][q] * (double)sW[q];
                acc[k] += a;
            }
        }
        __syncthreads();
    }
    if (mode == CGS_UPD_NORM) {
        const double s = block_sum256(nacc, red);
        if (tid == 0) partials[blockIdx.x] = s;
        return;
    }
#pragma unroll
    for (int k = 0; k < KPW; ++k) {
        const int v = wid + 4 * k;
        if (v < nv) {
            const double s = wave_sum64(acc[k]);
            if (lane == 0) partials[(long long)v * nchunks + blockIdx.x] = s;
        }
    }
}

// The same passes with the basis held in registers (as the single-problem
// k_cgs_reg): one element per thread and step, all NV basis loads of the
// element issued before its arithmetic (rows nv..NV-1 re-read row nv-1 with a
// zero coefficient), FP64 dots per thread reduced once per block.
template <typename T, int NV, int MODE>
__global__ __launch_bounds__(kB) void kb_cgs_reg(BTab t, const T* __restrict__ V, long long ntot, int nv,
                                                 const double* __restrict__ hin, T* __restrict__ w,
                                                 double* __restrict__ partials, int nchunks) {
    constexpr bool kDots = MODE != CGS_UPD_NORM;
    constexpr bool kUpd = MODE != CGS_DOT;
    __shared__ double red[4][kDots ? NV : 1];
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double h[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) h[v] = (kUpd && v < nv) ? hin[(long long)c.inst * M + v] : 0.0;
    double acc[kDots ? NV : 1];
#pragma unroll
    for (int v = 0; v < (kDots ? NV : 1); ++v) acc[v] = 0.0;
    double nacc = 0.0;
    for (long long i = c.b + tid; i < c.e; i += kB) {
        T wv = w[i];
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = V[(long long)(v < nv ? v : nv - 1) * ntot + i];
        __builtin_amdgcn_sched_barrier(0);   // all loads of the element ahead of its arithmetic
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
        const double s = block_sum256(nacc, &red[0][0]);
        if (tid == 0) partials[blockIdx.x] = s;
        return;
    }
    constexpr int kSpan = 64 / NV;
    const double s = wave_sum_scatter<kDots ? NV : 1>(acc, lane);
    if (lane % kSpan == 0) red[wid][lane / kSpan] = s;
    __syncthreads();
    if (tid < nv)
        partials[(long long)tid * nchunks + blockIdx.x] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// ---------------------------------------------------------------------------
// One-reduction Arnoldi step over the instances (the single-problem k_dg_*
// kernels, per chunk and per instance): the reduction pass writes per chunk
// the partial dots s (slots 0..), y (slots kDgMaxRows..), alpha and beta; one
// 1024-thread block per instance adds its chunks, closes column j-1 with its
// Givens step and forms the update coefficients; the update pass writes q_j
// and q~_{j+1} = (w - V y - q_j h_jj) / r_j.
// ---------------------------------------------------------------------------
enum { BD_S = 0, BD_Y = kDgMaxRows, BD_ALPHA = 2 * kDgMaxRows, BD_BETA = 2 * kDgMaxRows + 1,
       BD_SLOTS = 2 * kDgMaxRows + 2 };
constexpr int kBdCoef = 2 * M + 2;       // per instance: a[M], e[M], 1/r, c_w

template <typename T, int NV, bool W>
__global__ __launch_bounds__(kB) void kb_dg_dot(BTab t, const T* __restrict__ V, long long ntot, int j,
                                                double* __restrict__ partials, int nchunks) {
    constexpr int NA = W ? 2 * NV : NV;
    __shared__ double red[4][NA + 2];
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const T* q = V + (long long)j * ntot;
    const T* w = V + (long long)(j + 1) * ntot;
    const int last = j > 0 ? j - 1 : 0;      // rows past j - 1 re-read row j - 1 (row 0 when j = 0)
    double acc[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) acc[v] = 0.0;
    double aa = 0.0, ab = 0.0;
    for (long long i = c.b + tid; i < c.e; i += kB) {
        const T qv = q[i];
        const T wv = W ? w[i] : T(0);
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = V[(long long)(v < j ? v : last) * ntot + i];
        __builtin_amdgcn_sched_barrier(0);
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
    const double tsum = wave_sum_scatter<NA>(acc, lane);
    if (lane % kSpan == 0) red[wid][lane / kSpan] = tsum;
    const double ta = wave_sum64(aa);
    const double tb = W ? wave_sum64(ab) : 0.0;
    if (lane == 0) {
        red[wid][NA] = ta;
        red[wid][NA + 1] = tb;
    }
    __syncthreads();
    for (int o = tid; o < NA + 2; o += kB) {
        const double sum = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
        int slot = -1;
        if (o < NV) {
            if (o < j) slot = BD_S + o;
        } else if (o < NA) {
            if (o - NV < j) slot = BD_Y + (o - NV);
        } else if (o == NA) {
            slot = BD_ALPHA;
        } else if (W) {
            slot = BD_BETA;
        }
        if (slot >= 0) partials[(long long)slot * nchunks + blockIdx.x] = sum;
    }
}

struct BdArgs {
    double* H;
    double* Hraw;
    double* cs;
    double* sn;
    double* g;
    double* h1;
    double* rs;       // per instance: r_c, the norm of basis vector c before normalization
    double* coef;     // per instance: kBdCoef update coefficients
    double* scal;     // per instance: SB_WNORM <- r_j, SB_RES <- |g_j| after the Givens step
    int m;
};

__global__ __launch_bounds__(1024) void kb_dg_finish(BTab t, const double* __restrict__ partials, int nchunks, int j,
                                                     int with_w, BdArgs a) {
    const int inst = blockIdx.x;
    if (inactive(t, inst)) return;
    __shared__ double sums[BD_SLOTS];
    __shared__ double hp[M + 1], scs[M], ssn[M], pre[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int c0 = t.chunk_off[inst], c1 = t.chunk_off[inst + 1];
    for (int o = wid; o < BD_SLOTS; o += 16) {
        const bool need = o < BD_Y ? o < j : o < BD_ALPHA ? (with_w && o - BD_Y < j) : (o == BD_ALPHA || with_w);
        if (!need) continue;
        double acc = 0.0;
        for (int b = c0 + lane; b < c1; b += 64) acc += partials[(long long)o * nchunks + b];
        acc = wave_sum64(acc);
        if (lane == 0) sums[o] = acc;
    }
    const int m = a.m;
    double* H = a.H + (long long)inst * (M + 1) * M;
    double* Hraw = a.Hraw + (long long)inst * (M + 1) * M;
    double* cs = a.cs + (long long)inst * M;
    double* sn = a.sn + (long long)inst * M;
    double* g = a.g + (long long)inst * (M + 1);
    double* h1 = a.h1 + (long long)inst * M;
    double* rs = a.rs + (long long)inst * M;
    double* coef = a.coef + (long long)inst * kBdCoef;
    double* sc = a.scal + (long long)inst * S_STRIDE;
    for (int r = tid; r < j; r += 1024) {
        hp[r] = h1[r];
        scs[r] = cs[r];
        ssn[r] = sn[r];
    }
    if (tid == 1023 && j > 0) {
        pre[0] = rs[j - 1];
        pre[1] = g[j - 1];
    }
    __syncthreads();
    if (wid == 0) {
        const double sv = lane < j ? sums[BD_S + lane] : 0.0;
        const double yv = (with_w && lane < j) ? sums[BD_Y + lane] : 0.0;
        double ss = sv * sv, sy = sv * yv;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ss += __shfl_xor(ss, o, 64);
            sy += __shfl_xor(sy, o, 64);
        }
        const double r2 = sums[BD_ALPHA] - ss;
        const double r = r2 > 0.0 ? sqrt(r2) : (r2 != r2 ? r2 : 0.0);
        if (j > 0) {
            const double scl = pre[0];
            const double inv_scl = scl > 0.0 ? 1.0 / scl : 0.0;
            double h = 0.0;
            if (lane < j) h = hp[lane] + scl * sv;
            else if (lane == j) h = scl * r;
            if (lane <= j) {
                hp[lane] = h;
                Hraw[lane * m + (j - 1)] = h * inv_scl;
            }
        }
        if (with_w) {
            const double inv_r = r > 0.0 ? 1.0 / r : 0.0;
            const double hjj = (sums[BD_BETA] - sy) * inv_r;
            const double cw = hjj * inv_r;
            if (lane < j) {
                coef[lane] = sv;
                coef[M + lane] = yv - cw * sv;
            }
            if (lane == 0) {
                coef[2 * M] = inv_r;
                coef[2 * M + 1] = cw;
                pre[2] = hjj;
            }
        }
        if (lane == 0) pre[3] = r;
    }
    __syncthreads();
    if (with_w && tid < j) h1[tid] = sums[BD_Y + tid];
    if (tid != 0) return;
    const double r = pre[3];
    double res = 0.0;
    if (j == 0) {
        g[0] = r;
    } else {
        const int c = j - 1;
        double y = hp[0];
        for (int k = 0; k < c; ++k) {
            const double z = hp[k + 1];
            H[k * m + c] = scs[k] * y + ssn[k] * z;
            y = -ssn[k] * y + scs[k] * z;
        }
        const double z = hp[c + 1];
        const double rr = hypot(y, z);
        double cc = 1.0, snn = 0.0;
        if (rr > 0.0) {
            cc = y / rr;
            snn = z / rr;
        }
        cs[c] = cc;
        sn[c] = snn;
        H[c * m + c] = rr;
        H[(c + 1) * m + c] = 0.0;
        const double gc = pre[1];
        g[c + 1] = -snn * gc;
        g[c] = cc * gc;
        res = fabs(snn * gc);
    }
    rs[j] = r;
    if (with_w) h1[j] = pre[2];
    sc[SB_WNORM] = r;
    sc[SB_RES] = res;
}

template <typename T, int NV>
__global__ __launch_bounds__(kB) void kb_dg_update(BTab t, T* V, long long ntot, int j,
                                                   const double* __restrict__ coefs) {
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    const double* coef = coefs + (long long)c.inst * kBdCoef;
    T* q = V + (long long)j * ntot;
    T* w = V + (long long)(j + 1) * ntot;
    const int last = j > 0 ? j - 1 : 0;
    double ca[NV], ce[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ca[v] = v < j ? coef[v] : 0.0;
        ce[v] = v < j ? coef[M + v] : 0.0;
    }
    const double inv_r = coef[2 * M], cw = coef[2 * M + 1];
    for (long long i = c.b + threadIdx.x; i < c.e; i += kB) {
        const T qv = q[i], wv = w[i];
        T x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = V[(long long)(v < j ? v : last) * ntot + i];
        __builtin_amdgcn_sched_barrier(0);
        double sq = (double)qv, sw = (double)wv - cw * (double)qv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sq -= ca[v] * (double)x[v];
            sw -= ce[v] * (double)x[v];
        }
        q[i] = (T)(sq * inv_r);
        w[i] = (T)(sw * inv_r);
    }
}

// block (i, v): hout[i][v] = sum over instance i's chunks; after the last pass
// the Givens step of column j for instance i (one thread)
__global__ __launch_bounds__(kB) void kb_cgs_finish(BTab t, const double* __restrict__ partials, int nchunks,
                                                    double* hout, int mode, int j, int m, double* H, double* Hraw,
                                                    double* cs, double* sn, double* g, const double* h1,
                                                    const double* h2, double* scal) {
    __shared__ double red[4];
    const int i = blockIdx.x, v = blockIdx.y;
    if (inactive(t, i)) return;
    double acc = 0.0;
    const double* p = partials + (long long)v * nchunks;
    for (int b = t.chunk_off[i] + threadIdx.x; b < t.chunk_off[i + 1]; b += kB) acc += p[b];
    const double s = block_sum256(acc, red);
    if (threadIdx.x != 0) return;
    if (mode != CGS_UPD_NORM) {
        hout[(long long)i * M + v] = s;
        return;
    }
    const long long hb = (long long)i * (M + 1) * M;
    double* Hi = H + hb;
    double* Hr = Hraw + hb;
    double* ci = cs + (long long)i * M;
    double* si = sn + (long long)i * M;
    double* gi = g + (long long)i * (M + 1);
    double* sc = scal + (long long)i * S_STRIDE;
    for (int r = 0; r <= j; ++r) {
        const double h = h1[(long long)i * M + r] + h2[(long long)i * M + r];
        Hi[r * m + j] = h;
        Hr[r * m + j] = h;
    }
    const double nw = sqrt(s);
    Hi[(j + 1) * m + j] = nw;
    Hr[(j + 1) * m + j] = nw;
    for (int r = 0; r < j; ++r) {
        const double x = Hi[r * m + j], y = Hi[(r + 1) * m + j];
        Hi[r * m + j] = ci[r] * x + si[r] * y;
        Hi[(r + 1) * m + j] = -si[r] * x + ci[r] * y;
    }
    const double x = Hi[j * m + j], y = Hi[(j + 1) * m + j];
    const double rr = hypot(x, y);
    double cc = 1.0, ss = 0.0;
    if (rr > 0.0) {
        cc = x / rr;
        ss = y / rr;
    }
    ci[j] = cc;
    si[j] = ss;
    Hi[j * m + j] = rr;
    Hi[(j + 1) * m + j] = 0.0;
    gi[j + 1] = -ss * gi[j];
    gi[j] = cc * gi[j];
    sc[SB_WNORM] = nw;
    sc[SB_RES] = fabs(gi[j + 1]);
}

// g_i = (beta_i, 0, ...) for a new cycle
__global__ void kb_set_start(BTab t, double* g, const double* scal, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.ninst || inactive(t, i)) return;
    double* gi = g + (long long)i * (M + 1);
    gi[0] = scal[(long long)i * S_STRIDE + SB_BETA];
    for (int r = 1; r <= m; ++r) gi[r] = 0.0;
}

// y_i = R_i^{-1} g_i over the first k_i columns (k_i from kcnt; 0 skips)
__global__ void kb_backsolve(BTab t, const double* H, const double* g, const int* kcnt, int m, double* y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.ninst) return;
    const int k = kcnt[i];
    const double* Hi = H + (long long)i * (M + 1) * M;
    const double* gi = g + (long long)i * (M + 1);
    double* yi = y + (long long)i * M;
    for (int r = k - 1; r >= 0; --r) {
        double s = gi[r];
        for (int l = r + 1; l < k; ++l) s -= Hi[r * m + l] * yi[l];
        yi[r] = s / Hi[r * m + r];
    }
}

// x += Z y over each instance's k_i directions
template <typename T>
__global__ __launch_bounds__(kB) void kb_axpy_basis(BTab t, T* __restrict__ x, const T* __restrict__ Z, long long ntot,
                                                    const int* kcnt, const double* __restrict__ y) {
    const Chunk c = chunk_of(t);
    const int k = kcnt[c.inst];
    if (k == 0) return;
    const double* yi = y + (long long)c.inst * M;
    for (long long e = c.b + threadIdx.x; e < c.e; e += kB) {
        double s = (double)x[e];
        for (int v = 0; v < k; ++v) s += yi[v] * (double)Z[(long long)v * ntot + e];
        x[e] = (T)s;
    }
}

// z = v (no preconditioner), v normalised by div_i first
template <typename T>
__global__ __launch_bounds__(kB) void kb_normalize_copy(BTab t, T* __restrict__ v, const double* __restrict__ scal,
                                                        int which, T* __restrict__ z) {
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    if (which < 0) {                      // copy only (the one-reduction step keeps V_j as it is)
        for (long long e = c.b + threadIdx.x; e < c.e; e += kB) z[e] = v[e];
        return;
    }
    const double d = scal[(long long)c.inst * S_STRIDE + which];
    for (long long e = c.b + threadIdx.x; e < c.e; e += kB) {
        const T o = (T)((double)v[e] / d);
        v[e] = o;
        z[e] = o;
    }
}

// out = a x + b y for active instances
template <typename T>
__global__ __launch_bounds__(kB) void kb_lincomb(BTab t, T* __restrict__ o, const T* __restrict__ x,
                                                 const T* __restrict__ y, double a, double b) {
    const Chunk c = chunk_of(t);
    if (inactive(t, c.inst)) return;
    for (long long e = c.b + threadIdx.x; e < c.e; e += kB) o[e] = (T)(a * (double)x[e] + b * (double)y[e]);
}

template <typename T>
__global__ __launch_bounds__(kB) void kb_zero(BTab t, T* __restrict__ x) {
    const Chunk c = chunk_of(t);
    for (long long e = c.b + threadIdx.x; e < c.e; e += kB) x[e] = T(0);
}

// ---- per-instance decisions on the device (the captured-graph cycle) ----
// Instance state of a lockstep GMRES solve kept in device memory so that a
// whole restart cycle runs without the host: act (working), in_cycle (worked
// in this cycle), conv, iters, kcnt (columns of this cycle), tol and bnorm
// (relative tolerance and ||rhs||), flags[0] = any instance active after the
// cycle, flags[1] = a non-finite norm was met.
struct BDev {
    int* act;
    int* in_cycle;
    int* conv;
    int* iters;
    int* kcnt;
    const double* tol;
    double* bnorm;
    int* flags;
};

// start of a solve: iteration counts and convergence cleared, ||rhs|| taken
// from the cycle-start norm; a zero right-hand side is solved, a non-finite
// one flagged
__global__ void kb_dev_begin(int ni, BDev d, const double* __restrict__ scal) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) d.flags[1] = 0;
    if (i >= ni) return;
    d.conv[i] = 0;
    d.iters[i] = 0;
    d.kcnt[i] = 0;
    if (!d.act[i]) return;
    const double b = scal[(long long)i * S_STRIDE + SB_BETA];
    d.bnorm[i] = b;
    if (!isfinite(b)) {
        d.flags[1] = 1;
        d.act[i] = 0;
    } else if (b == 0.0) {
        d.act[i] = 0;
        d.conv[i] = 1;
    }
}

__global__ void kb_dev_cycle_begin(int ni, BDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    d.in_cycle[i] = d.act[i];
    d.kcnt[i] = 0;
}

// column col of every working instance is final: count it and stop the
// instances that are done (converged, exact, out of iterations or, with
// last_col, at the end of the cycle)
__global__ void kb_dev_close(int ni, BDev d, const double* __restrict__ scal, int col, int max_iters, int last_col) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || !d.act[i]) return;
    const double r = scal[(long long)i * S_STRIDE + SB_WNORM];
    const double res = scal[(long long)i * S_STRIDE + SB_RES];
    if (!isfinite(r) || !isfinite(res)) {
        d.flags[1] = 1;
        d.act[i] = 0;
        return;
    }
    d.kcnt[i] = col + 1;
    const int it = d.iters[i] + 1;
    d.iters[i] = it;
    const bool ok = res <= d.tol[i] * d.bnorm[i];
    if (ok || r == 0.0 || it >= max_iters || (last_col && col + 1 == last_col)) {
        d.act[i] = 0;
        d.conv[i] = ok ? 1 : 0;
    }
}

// after a one-reduction cycle: the instances that ended it unconverged with
// iterations left restart
__global__ void kb_dev_restart_select(int ni, BDev d, int m, int max_iters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    d.act[i] = (d.in_cycle[i] && !d.conv[i] && d.iters[i] < max_iters && d.kcnt[i] == m) ? 1 : 0;
}

// after the restart residual: r = 0 ends an instance
__global__ void kb_dev_beta_zero(int ni, BDev d, const double* __restrict__ scal) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni || !d.act[i]) return;
    const double b = scal[(long long)i * S_STRIDE + SB_BETA];
    if (!isfinite(b)) {
        d.flags[1] = 1;
        d.act[i] = 0;
    } else if (b == 0.0) {
        d.act[i] = 0;
        d.conv[i] = 1;
    }
}

// flags[0] = some instance still works (one block)
__global__ __launch_bounds__(256) void kb_dev_any(int ni, BDev d) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < ni; i += 256)
        if (d.act[i]) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) d.flags[0] = any;
}

}  // namespace
}  // namespace jfnk

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace jfnk;

struct jfnk_batch {
    int ninst = 0, max_m = 0;
    int W = 2;                  // stencil half-width of every instance (dd_p = 3: 4)
    hipStream_t stream = nullptr;
    std::vector<jfnk_problem> probs;
    std::vector<Geo> geos;
    std::vector<long long> voff, poff, noff;
    std::vector<int> tile_off[3], tiles_x[3], pblk_off, eblk_off, chunk_off;
    long long ntot = 0, ptot = 0, netot = 0;
    int nchunks = 0;
    int tune[6] = {1, 1, 1, 1, 1, 1};
    // device tables
    Geo* d_geos = nullptr;
    long long *d_voff = nullptr, *d_poff = nullptr, *d_noff = nullptr;
    int *d_tile_off[3] = {nullptr, nullptr, nullptr}, *d_tiles_x[3] = {nullptr, nullptr, nullptr};
    int *d_pblk_off = nullptr, *d_eblk_off = nullptr, *d_chunk_off = nullptr;
    int* d_active = nullptr;
    int* d_kcnt = nullptr;
    // vectors
    float *V32 = nullptr, *Z32 = nullptr, *u32 = nullptr, *b32 = nullptr, *x32 = nullptr, *t32 = nullptr,
          *nu32 = nullptr;
    double *f64 = nullptr, *R64 = nullptr;
    double *bg64 = nullptr;
    float* bg32 = nullptr;
    // per-instance scalars
    double *H = nullptr, *Hraw = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *h1 = nullptr,
           *h2 = nullptr, *scal = nullptr, *outv = nullptr;
    double* coef = nullptr;     // one-reduction step: update coefficients per instance
    double* partials = nullptr;
    double* hscal = nullptr;    // pinned: ninst * S_STRIDE
    int* hflags = nullptr;      // pinned: ninst
    // device-side instance state of the captured cycle (see BDev)
    int *d_incycle = nullptr, *d_conv = nullptr, *d_iters = nullptr, *d_dflags = nullptr;
    double *d_tol = nullptr, *d_bnorm = nullptr;
    int* hdflags = nullptr;     // pinned: 2 (any, non-finite) per cycle
    double* htol = nullptr;     // pinned: ninst
    int* hres = nullptr;        // pinned: 2 ninst (iters, conv)
    hipStream_t cap_stream = nullptr;   // capture stream (a graph cannot be captured on the null stream)
    hipGraphExec_t cycle_exec = nullptr;
    int cyc_key[8] = {-1, -1, -1, -1, -1, -1, -1, -1};   // the options the captured cycle was built for
};

namespace {

BTab tab(jfnk_batch* b, int variant, bool masked) {
    BTab t;
    t.ninst = b->ninst;
    t.geos = b->d_geos;
    t.voff = b->d_voff;
    t.poff = b->d_poff;
    t.noff = b->d_noff;
    t.tile_off = b->d_tile_off[variant];
    t.tiles_x = b->d_tiles_x[variant];
    t.pblk_off = b->d_pblk_off;
    t.eblk_off = b->d_eblk_off;
    t.chunk_off = b->d_chunk_off;
    t.active = masked ? b->d_active : nullptr;
    return t;
}

int ntiles(jfnk_batch* b, int variant) { return b->tile_off[variant][b->ninst]; }

template <typename T>
hipError_t b_apply_F(jfnk_batch* b, const T* u, const T* f, T* out, int what, int var = -1) {
    if (var < 0) var = b->tune[0 * 2 + (sizeof(T) == 4)];
    const BTab t = tab(b, var, false);
    const dim3 grid(ntiles(b, var));
    if (b->W == 4) {
        if (var == 0) hipLaunchKernelGGL((kb_apply_F<T, 4, 4>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
        else if (var == 2) hipLaunchKernelGGL((kb_apply_F<T, 16, 4>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
        else hipLaunchKernelGGL((kb_apply_F<T, 8, 4>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
    } else {
        if (var == 0) hipLaunchKernelGGL((kb_apply_F<T, 4, 2>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
        else if (var == 2) hipLaunchKernelGGL((kb_apply_F<T, 16, 2>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
        else hipLaunchKernelGGL((kb_apply_F<T, 8, 2>), grid, dim3(kB), 0, b->stream, t, u, f, out, what);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t b_jv(jfnk_batch* b, const T* u, const T* v, const double* eps, T* out, int var) {
    // the tile table of the height the kernel really uses
    if (sizeof(T) == 8 && b->W == 4) var = 0;
    else if (sizeof(T) == 8 && var == 2) var = 1;
    const BTab t = tab(b, var, true);
    const dim3 grid(ntiles(b, var));
    if (b->W == 4) {
        if (var == 0) hipLaunchKernelGGL((kb_jv<T, 4, 4>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
        else if (var == 2) hipLaunchKernelGGL((kb_jv<T, 16, 4>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
        else hipLaunchKernelGGL((kb_jv<T, 8, 4>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
    } else {
        if (var == 0) hipLaunchKernelGGL((kb_jv<T, 4, 2>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
        else if (var == 2) hipLaunchKernelGGL((kb_jv<T, 16, 2>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
        else hipLaunchKernelGGL((kb_jv<T, 8, 2>), grid, dim3(kB), 0, b->stream, t, u, v, eps, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t b_pc_sweep(jfnk_batch* b, const T* u, const T* nu, const T* r, const T* zin, T* zout, int var) {
    static_assert(sizeof(T) == 4, "the ensemble's preconditioner sweeps run in FP32");
    const BTab t = tab(b, var, true);
    const dim3 grid(ntiles(b, var));
    if (b->W == 4) {
        if (var == 0) hipLaunchKernelGGL((kb_pc_sweep<T, 4, 4>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
        else if (var == 2)
            hipLaunchKernelGGL((kb_pc_sweep<T, 16, 4>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
        else hipLaunchKernelGGL((kb_pc_sweep<T, 8, 4>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
    } else {
        if (var == 0) hipLaunchKernelGGL((kb_pc_sweep<T, 4, 2>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
        else if (var == 2)
            hipLaunchKernelGGL((kb_pc_sweep<T, 16, 2>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
        else hipLaunchKernelGGL((kb_pc_sweep<T, 8, 2>), grid, dim3(kB), 0, b->stream, t, u, nu, r, zin, zout);
    }
    return hipGetLastError();
}

// frozen viscosity on every instance's ring-W grid; z = v / d of the active instances
void b_frozen_nu(jfnk_batch* b, const BTab& t, const float* u) {
    const dim3 grid(b->eblk_off[b->ninst]);
    if (b->W == 4) hipLaunchKernelGGL((kb_frozen_nu<float, 4>), grid, dim3(kB), 0, b->stream, t, u, b->nu32);
    else hipLaunchKernelGGL((kb_frozen_nu<float, 2>), grid, dim3(kB), 0, b->stream, t, u, b->nu32);
}
void b_pc_diag(jfnk_batch* b, const BTab& t, float* vj, const double* div, float* z) {
    const dim3 grid(b->pblk_off[b->ninst]);
    const float* nu = b->nu32;
    if (b->W == 4) hipLaunchKernelGGL((kb_pc_diag<float, 4>), grid, dim3(kB), 0, b->stream, t, nu, vj, div, z);
    else hipLaunchKernelGGL((kb_pc_diag<float, 2>), grid, dim3(kB), 0, b->stream, t, nu, vj, div, z);
}

// per-instance squared norms of x into out[i * stride], with a finishing mode
template <typename T>
int b_norm2(jfnk_batch* b, const T* x, double* out, int stride, int mode, bool masked, double sqrt_eps = 0.0) {
    const BTab t = tab(b, 1, masked);
    hipLaunchKernelGGL((kb_norm2<T>), dim3(b->nchunks), dim3(kB), 0, b->stream, t, x, b->partials);
    JFNK_HIP(hipGetLastError());
    hipLaunchKernelGGL(kb_finish, dim3(b->ninst), dim3(kB), 0, b->stream, t, (const double*)b->partials, out, stride,
                       mode, b->scal, sqrt_eps);
    JFNK_HIP(hipGetLastError());
    return JFNK_OK;
}

template <typename T, int NV>
hipError_t launch_kb_cgs_reg_nv(const BTab& t, const T* V, long long ntot, int nv, const double* hin, T* w,
                                double* partials, int nchunks, int mode, hipStream_t s) {
    const dim3 grid(nchunks);
    if (mode == CGS_DOT)
        hipLaunchKernelGGL((kb_cgs_reg<T, NV, CGS_DOT>), grid, dim3(kB), 0, s, t, V, ntot, nv, hin, w, partials,
                           nchunks);
    else if (mode == CGS_UPD_DOT)
        hipLaunchKernelGGL((kb_cgs_reg<T, NV, CGS_UPD_DOT>), grid, dim3(kB), 0, s, t, V, ntot, nv, hin, w, partials,
                           nchunks);
    else
        hipLaunchKernelGGL((kb_cgs_reg<T, NV, CGS_UPD_NORM>), grid, dim3(kB), 0, s, t, V, ntot, nv, hin, w,
                           partials, nchunks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kb_cgs_reg(const BTab& t, const T* V, long long ntot, int nv, const double* hin, T* w,
                             double* partials, int nchunks, int mode, hipStream_t s) {
    if (nv <= 8) return launch_kb_cgs_reg_nv<T, 8>(t, V, ntot, nv, hin, w, partials, nchunks, mode, s);
    if (nv <= 16) return launch_kb_cgs_reg_nv<T, 16>(t, V, ntot, nv, hin, w, partials, nchunks, mode, s);
    return launch_kb_cgs_reg_nv<T, 32>(t, V, ntot, nv, hin, w, partials, nchunks, mode, s);
}

template <typename T>
int b_cgs(jfnk_batch* b, int nv, int mode, const double* hin, T* w, double* hout, int j, int m) {
    const BTab t = tab(b, 1, true);
    const long long ntot = b->ntot;
    const dim3 grid(b->nchunks);
    if (nv <= 32)
        JFNK_HIP(launch_kb_cgs_reg<T>(t, (const T*)b->V32, ntot, nv, hin, w, b->partials, b->nchunks, mode,
                                      b->stream));
    else
        hipLaunchKernelGGL((kb_cgs<T, 64>), grid, dim3(kB), 0, b->stream, t, (const T*)b->V32, ntot, nv, hin, w,
                           b->partials, b->nchunks, mode);
    JFNK_HIP(hipGetLastError());
    const int nacc = mode == CGS_UPD_NORM ? 1 : nv;
    hipLaunchKernelGGL(kb_cgs_finish, dim3(b->ninst, nacc), dim3(kB), 0, b->stream, t, (const double*)b->partials,
                       b->nchunks, hout, mode, j, m, b->H, b->Hraw, b->cs, b->sn, b->g, (const double*)b->h1,
                       (const double*)b->h2, b->scal);
    JFNK_HIP(hipGetLastError());
    return JFNK_OK;
}

int b_read_scal(jfnk_batch* b) {
    JFNK_HIP(hipMemcpyAsync(b->hscal, b->scal, (size_t)b->ninst * S_STRIDE * sizeof(double), hipMemcpyDeviceToHost,
                            b->stream));
    JFNK_HIP(hipStreamSynchronize(b->stream));
    return JFNK_OK;
}

// The pinned flag buffer is reused by the next call: wait for the copy.
int b_set_active(jfnk_batch* b, const std::vector<int>& act) {
    for (int i = 0; i < b->ninst; ++i) b->hflags[i] = act[i];
    JFNK_HIP(hipMemcpyAsync(b->d_active, b->hflags, b->ninst * sizeof(int), hipMemcpyHostToDevice, b->stream));
    JFNK_HIP(hipStreamSynchronize(b->stream));
    return JFNK_OK;
}

int b_set_kcnt(jfnk_batch* b, const std::vector<int>& k) {
    for (int i = 0; i < b->ninst; ++i) b->hflags[i] = k[i];
    JFNK_HIP(hipMemcpyAsync(b->d_kcnt, b->hflags, b->ninst * sizeof(int), hipMemcpyHostToDevice, b->stream));
    JFNK_HIP(hipStreamSynchronize(b->stream));   // hflags is reused right after
    return JFNK_OK;
}

// Start of both ensemble GMRES forms over the instances with act[i] = 1: x = 0,
// frozen coefficients, ||u_i||^2, V_0 = rhs and beta_i = ||rhs_i|| (bnorm, res);
// instances with beta_i = 0 are done (converged).
int b_gmres_begin(jfnk_batch* b, const float* u, const float* rhs, float* x, const jfnk_gmres_opts& o,
                  std::vector<int>& act, std::vector<int>& conv, std::vector<double>& bnorm,
                  std::vector<double>& res) {
    const int ni = b->ninst;
    hipStream_t s = b->stream;
    int rc;
    if ((rc = b_set_active(b, act))) return rc;
    {
        const BTab t = tab(b, 1, false);
        hipLaunchKernelGGL((kb_zero<float>), dim3(b->nchunks), dim3(kB), 0, s, t, x);
        JFNK_HIP(hipGetLastError());
        if (o.pc == JFNK_PC_PHYSICS) {
            const BTab ta = tab(b, 1, true);
            b_frozen_nu(b, ta, u);
            JFNK_HIP(hipGetLastError());
        }
    }
    if ((rc = b_norm2<float>(b, u, b->scal + SB_UNORM2, S_STRIDE, FIN_STORE, true))) return rc;
    JFNK_HIP(hipMemcpyAsync(b->V32, rhs, b->ntot * sizeof(float), hipMemcpyDeviceToDevice, s));
    if ((rc = b_norm2<float>(b, b->V32, b->outv, 1, FIN_BETA, true))) return rc;
    if ((rc = b_read_scal(b))) return rc;
    bnorm.assign(ni, 0.0);
    res.assign(ni, 0.0);
    for (int i = 0; i < ni; ++i) {
        if (!act[i]) continue;
        bnorm[i] = b->hscal[(long long)i * S_STRIDE + SB_BETA];
        if (!std::isfinite(bnorm[i])) {
            set_error("non-finite right-hand side norm in the batch");
            return JFNK_ERR_NONFINITE;
        }
        res[i] = bnorm[i];
        if (bnorm[i] == 0.0) {
            act[i] = 0;
            conv[i] = 1;
        }
    }
    return JFNK_OK;
}

// Restart of the active instances (d_active set): the true residual
// r_i = rhs_i - J_i x_i into V_0 and beta_i = ||r_i||; r_i = 0 ends instance i.
int b_restart_residual(jfnk_batch* b, const float* u, const float* rhs, const float* x, std::vector<int>& act,
                       std::vector<int>& conv) {
    const double sqrt_eps = std::sqrt(1.1920928955078125e-07);
    hipStream_t s = b->stream;
    int rc;
    const BTab tr = tab(b, 1, true);
    if ((rc = b_norm2<float>(b, x, b->scal + SB_VNORM2, S_STRIDE, FIN_EPS, true, sqrt_eps))) return rc;
    JFNK_HIP(b_jv<float>(b, u, x, b->scal + SB_EPS, b->V32, b->tune[1 * 2 + 1]));
    hipLaunchKernelGGL((kb_lincomb<float>), dim3(b->nchunks), dim3(kB), 0, s, tr, b->V32, rhs, b->V32, 1.0, -1.0);
    JFNK_HIP(hipGetLastError());
    if ((rc = b_norm2<float>(b, b->V32, b->outv, 1, FIN_BETA, true))) return rc;
    if ((rc = b_read_scal(b))) return rc;
    for (int i = 0; i < b->ninst; ++i)
        if (act[i] && b->hscal[(long long)i * S_STRIDE + SB_BETA] == 0.0) {
            act[i] = 0;
            conv[i] = 1;
        }
    return JFNK_OK;
}

template <typename T>
hipError_t launch_kb_dg_dot(jfnk_batch* b, const BTab& t, int j, bool with_w) {
    const dim3 grid(b->nchunks);
    const float* V = (const float*)b->V32;
    if (with_w) {
        if (j <= 8)
            hipLaunchKernelGGL((kb_dg_dot<T, 8, true>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j, b->partials,
                               b->nchunks);
        else if (j <= 16)
            hipLaunchKernelGGL((kb_dg_dot<T, 16, true>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j, b->partials,
                               b->nchunks);
        else
            hipLaunchKernelGGL((kb_dg_dot<T, 32, true>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j, b->partials,
                               b->nchunks);
    } else {
        if (j <= 8)
            hipLaunchKernelGGL((kb_dg_dot<T, 8, false>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j, b->partials,
                               b->nchunks);
        else if (j <= 16)
            hipLaunchKernelGGL((kb_dg_dot<T, 16, false>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j,
                               b->partials, b->nchunks);
        else
            hipLaunchKernelGGL((kb_dg_dot<T, 32, false>), grid, dim3(kB), 0, b->stream, t, V, b->ntot, j,
                               b->partials, b->nchunks);
    }
    return hipGetLastError();
}

// reduction (and, with w, the update) of the one-reduction step j for the
// active instances; r_j and |g_j| land in scal (SB_WNORM, SB_RES)
int b_dg(jfnk_batch* b, int j, bool with_w, int m) {
    if (j < 0 || j >= kDgMaxRows) {
        set_error("the one-reduction step handles fewer than 32 basis vectors");
        return JFNK_ERR_ARG;
    }
    const BTab t = tab(b, 1, true);
    JFNK_HIP(launch_kb_dg_dot<float>(b, t, j, with_w));
    BdArgs a;
    a.H = b->H;
    a.Hraw = b->Hraw;
    a.cs = b->cs;
    a.sn = b->sn;
    a.g = b->g;
    a.h1 = b->h1;
    a.rs = b->h2;             // CGS2's second-pass coefficients are unused here
    a.coef = b->coef;
    a.scal = b->scal;
    a.m = m;
    hipLaunchKernelGGL(kb_dg_finish, dim3(b->ninst), dim3(1024), 0, b->stream, t, (const double*)b->partials,
                       b->nchunks, j, with_w ? 1 : 0, a);
    JFNK_HIP(hipGetLastError());
    if (!with_w) return JFNK_OK;
    float* V = b->V32;
    if (j <= 8)
        hipLaunchKernelGGL((kb_dg_update<float, 8>), dim3(b->nchunks), dim3(kB), 0, b->stream, t, V, b->ntot, j,
                           (const double*)b->coef);
    else if (j <= 16)
        hipLaunchKernelGGL((kb_dg_update<float, 16>), dim3(b->nchunks), dim3(kB), 0, b->stream, t, V, b->ntot, j,
                           (const double*)b->coef);
    else
        hipLaunchKernelGGL((kb_dg_update<float, 32>), dim3(b->nchunks), dim3(kB), 0, b->stream, t, V, b->ntot, j,
                           (const double*)b->coef);
    JFNK_HIP(hipGetLastError());
    return JFNK_OK;
}

// b_gmres with the one-reduction Arnoldi step: column j-1 of an instance is
// closed at iteration j (or by the closing reduction at the end of a cycle),
// so its convergence is known one iteration later; the basis vectors stay
// unnormalized until then.
int b_gmres_one_reduction(jfnk_batch* b, const float* u, const float* rhs, float* x, const std::vector<int>& act0,
                          const std::vector<double>& tol, const jfnk_gmres_opts& o, std::vector<int>& iters,
                          std::vector<int>& conv) {
    const int ni = b->ninst, m = o.m;
    const long long ntot = b->ntot;
    const int max_iters = o.max_iters > 0 ? o.max_iters : m * o.max_restarts;
    const double sqrt_eps = std::sqrt(1.1920928955078125e-07);
    hipStream_t s = b->stream;
    std::vector<int> act = act0;
    iters.assign(ni, 0);
    conv.assign(ni, 0);
    int rc;
    std::vector<double> bnorm, res;
    if ((rc = b_gmres_begin(b, u, rhs, x, o, act, conv, bnorm, res))) return rc;
    const BTab tall = tab(b, 1, false);
    // after the reduction that closed column `col` of every active instance:
    // count it and stop the instances that are done
    auto close_column = [&](int col, std::vector<int>& kcnt, bool& any) -> int {
        if ((rc = b_read_scal(b))) return rc;
        any = false;
        for (int i = 0; i < ni; ++i) {
            if (!act[i]) continue;
            const double r = b->hscal[(long long)i * S_STRIDE + SB_WNORM];
            res[i] = b->hscal[(long long)i * S_STRIDE + SB_RES];
            if (!std::isfinite(r) || !std::isfinite(res[i])) {
                set_error("non-finite Krylov norm in the batch");
                return JFNK_ERR_NONFINITE;
            }
            kcnt[i] = col + 1;
            iters[i]++;
            if (res[i] <= tol[i] * bnorm[i] || r == 0.0 || iters[i] >= max_iters || col + 1 == m) {
                act[i] = 0;
                conv[i] = res[i] <= tol[i] * bnorm[i] ? 1 : 0;
            } else {
                any = true;
            }
        }
        return JFNK_OK;
    };
    while (true) {
        if (std::none_of(act.begin(), act.end(), [](int a) { return a; })) break;
        if ((rc = b_set_active(b, act))) return rc;
        const BTab ta = tab(b, 1, true);
        hipLaunchKernelGGL(kb_set_start, dim3((ni + 255) / 256), dim3(256), 0, s, ta, b->g, (const double*)b->scal, m);
        JFNK_HIP(hipGetLastError());
        std::vector<int> kcnt(ni, 0);
        const std::vector<int> in_cycle = act;
        bool closed_last = false;
        for (int j = 0; j < m; ++j) {
            float* Vj = b->V32 + (long long)j * ntot;
            float* Vn = b->V32 + (long long)(j + 1) * ntot;
            float* Zj = b->Z32 + (long long)j * ntot;
            // z_j = M^-1 q~_j (q~_j not normalized)
            if (o.pc == JFNK_PC_PHYSICS) {
                float* bufs[2] = {Zj, b->t32};
                int cur = (o.sweeps % 2 == 0) ? 0 : 1;
                b_pc_diag(b, ta, Vj, nullptr, bufs[cur]);
                JFNK_HIP(hipGetLastError());
                for (int sw = 0; sw < o.sweeps; ++sw) {
                    JFNK_HIP(b_pc_sweep<float>(b, u, b->nu32, Vj, bufs[cur], bufs[1 - cur], b->tune[2 * 2 + 1]));
                    cur = 1 - cur;
                }
            } else {
                hipLaunchKernelGGL((kb_normalize_copy<float>), dim3(b->nchunks), dim3(kB), 0, s, ta, Vj,
                                   (const double*)b->scal, -1, Zj);
                JFNK_HIP(hipGetLastError());
            }
            if ((rc = b_norm2<float>(b, Zj, b->scal + SB_VNORM2, S_STRIDE, FIN_EPS, true, sqrt_eps))) return rc;
            JFNK_HIP(b_jv<float>(b, u, Zj, b->scal + SB_EPS, Vn, b->tune[1 * 2 + 1]));
            if ((rc = b_dg(b, j, true, m))) return rc;
            if (j == 0) continue;                       // no column closed yet
            bool any = false;
            if ((rc = close_column(j - 1, kcnt, any))) return rc;
            if (!any) {
                closed_last = true;
                break;
            }
            if ((rc = b_set_active(b, act))) return rc;
        }
        if (!closed_last) {
            // column m-1 of the instances still working: closing reduction over q~_m
            if ((rc = b_set_active(b, act))) return rc;
            if ((rc = b_dg(b, m, false, m))) return rc;
            bool any = false;
            if ((rc = close_column(m - 1, kcnt, any))) return rc;
        }
        // solution update of every instance that worked in this cycle
        if ((rc = b_set_kcnt(b, kcnt))) return rc;
        hipLaunchKernelGGL(kb_backsolve, dim3((ni + 63) / 64), dim3(64), 0, s, tall, (const double*)b->H,
                           (const double*)b->g, (const int*)b->d_kcnt, m, b->y);
        JFNK_HIP(hipGetLastError());
        hipLaunchKernelGGL((kb_axpy_basis<float>), dim3(b->nchunks), dim3(kB), 0, s, tall, x, (const float*)b->Z32,
                           ntot, (const int*)b->d_kcnt, (const double*)b->y);
        JFNK_HIP(hipGetLastError());
        // instances that ended the cycle unconverged with iterations left restart from the true residual
        for (int i = 0; i < ni; ++i)
            if (in_cycle[i] && !conv[i] && iters[i] < max_iters && kcnt[i] == m) act[i] = 1;
        if (std::none_of(act.begin(), act.end(), [](int a) { return a; })) break;
        if ((rc = b_set_active(b, act))) return rc;
        if ((rc = b_restart_residual(b, u, rhs, x, act, conv))) return rc;
    }
    JFNK_HIP(hipStreamSynchronize(s));
    return JFNK_OK;
}

BDev bdev(jfnk_batch* b) {
    return {b->d_active, b->d_incycle, b->d_conv, b->d_iters, b->d_kcnt, b->d_tol, b->d_bnorm, b->d_dflags};
}

// One restart cycle of the lockstep FGMRES(m) with every decision on the
// device: m iterations of the preconditioner, Jv and Arnoldi step (each launch
// masked by the instances still working), column closes, the solution update
// over the columns each instance counted, the choice of the instances that
// restart, their true residual, and the flags the host reads after the cycle.
// Nothing here synchronises, allocates or clears memory with a memset, so the
// sequence can be captured as a graph and replayed.
int b_enqueue_cycle(jfnk_batch* b, const float* u, const float* rhs, float* x, const jfnk_gmres_opts& o,
                    int max_iters) {
    const int ni = b->ninst, m = o.m;
    const long long ntot = b->ntot;
    const double sqrt_eps = std::sqrt(1.1920928955078125e-07);
    const bool onered = o.ortho == JFNK_ORTHO_ONE_REDUCTION && m < kDgMaxRows;
    hipStream_t s = b->stream;
    const BDev d = bdev(b);
    const dim3 g1((ni + 255) / 256), b1(256);
    int rc;
    const BTab ta = tab(b, 1, true), tall = tab(b, 1, false);
    hipLaunchKernelGGL(kb_set_start, g1, b1, 0, s, ta, b->g, (const double*)b->scal, m);
    hipLaunchKernelGGL(kb_dev_cycle_begin, g1, b1, 0, s, ni, d);
    JFNK_HIP(hipGetLastError());
    for (int j = 0; j < m; ++j) {
        float* Vj = b->V32 + (long long)j * ntot;
        float* Vn = b->V32 + (long long)(j + 1) * ntot;
        float* Zj = b->Z32 + (long long)j * ntot;
        const int which = onered ? -1 : (j == 0 ? SB_BETA : SB_WNORM);
        if (o.pc == JFNK_PC_PHYSICS) {
            float* bufs[2] = {Zj, b->t32};
            int cur = (o.sweeps % 2 == 0) ? 0 : 1;
            b_pc_diag(b, ta, Vj, onered ? (const double*)nullptr : (const double*)(b->scal + which), bufs[cur]);
            JFNK_HIP(hipGetLastError());
            for (int sw = 0; sw < o.sweeps; ++sw) {
                JFNK_HIP(b_pc_sweep<float>(b, u, b->nu32, Vj, bufs[cur], bufs[1 - cur], b->tune[2 * 2 + 1]));
                cur = 1 - cur;
            }
        } else {
            hipLaunchKernelGGL((kb_normalize_copy<float>), dim3(b->nchunks), dim3(kB), 0, s, ta, Vj,
                               (const double*)b->scal, which, Zj);
            JFNK_HIP(hipGetLastError());
        }
        if ((rc = b_norm2<float>(b, Zj, b->scal + SB_VNORM2, S_STRIDE, FIN_EPS, true, sqrt_eps))) return rc;
        JFNK_HIP(b_jv<float>(b, u, Zj, b->scal + SB_EPS, Vn, b->tune[1 * 2 + 1]));
        if (onered) {
            if ((rc = b_dg(b, j, true, m))) return rc;
            if (j > 0) hipLaunchKernelGGL(kb_dev_close, g1, b1, 0, s, ni, d, (const double*)b->scal, j - 1, max_iters, m);
        } else {
            if ((rc = b_cgs<float>(b, j + 1, CGS_DOT, nullptr, Vn, b->h1, j, m))) return rc;
            if ((rc = b_cgs<float>(b, j + 1, CGS_UPD_DOT, b->h1, Vn, b->h2, j, m))) return rc;
            if ((rc = b_cgs<float>(b, j + 1, CGS_UPD_NORM, b->h2, Vn, b->outv, j, m))) return rc;
            hipLaunchKernelGGL(kb_dev_close, g1, b1, 0, s, ni, d, (const double*)b->scal, j, max_iters, 0);
        }
        JFNK_HIP(hipGetLastError());
    }
    if (onered) {
        // column m-1 of the instances still working: closing reduction over q~_m
        if ((rc = b_dg(b, m, false, m))) return rc;
        hipLaunchKernelGGL(kb_dev_close, g1, b1, 0, s, ni, d, (const double*)b->scal, m - 1, max_iters, m);
        JFNK_HIP(hipGetLastError());
    }
    // solution update of every instance that worked in this cycle
    hipLaunchKernelGGL(kb_backsolve, dim3((ni + 63) / 64), dim3(64), 0, s, tall, (const double*)b->H,
                       (const double*)b->g, (const int*)b->d_kcnt, m, b->y);
    hipLaunchKernelGGL((kb_axpy_basis<float>), dim3(b->nchunks), dim3(kB), 0, s, tall, x, (const float*)b->Z32, ntot,
                       (const int*)b->d_kcnt, (const double*)b->y);
    JFNK_HIP(hipGetLastError());
    if (onered) hipLaunchKernelGGL(kb_dev_restart_select, g1, b1, 0, s, ni, d, m, max_iters);
    // restart of the instances still working: true residual r = rhs - J x into V_0
    const BTab tr = tab(b, 1, true);
    if ((rc = b_norm2<float>(b, x, b->scal + SB_VNORM2, S_STRIDE, FIN_EPS, true, sqrt_eps))) return rc;
    JFNK_HIP(b_jv<float>(b, u, x, b->scal + SB_EPS, b->V32, b->tune[1 * 2 + 1]));
    hipLaunchKernelGGL((kb_lincomb<float>), dim3(b->nchunks), dim3(kB), 0, s, tr, b->V32, rhs, b->V32, 1.0, -1.0);
    JFNK_HIP(hipGetLastError());
    if ((rc = b_norm2<float>(b, b->V32, b->outv, 1, FIN_BETA, true))) return rc;
    hipLaunchKernelGGL(kb_dev_beta_zero, g1, b1, 0, s, ni, d, (const double*)b->scal);
    hipLaunchKernelGGL(kb_dev_any, dim3(1), dim3(256), 0, s, ni, d);
    JFNK_HIP(hipGetLastError());
    JFNK_HIP(hipMemcpyAsync(b->hdflags, b->d_dflags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    return JFNK_OK;
}

// Lockstep FGMRES(m) with device-side decisions: one captured graph per
// restart cycle, replayed until no instance works; the host synchronises once
// per cycle (to read whether any instance is left) instead of twice per
// iteration.  Same arithmetic and results as b_gmres.
int b_gmres_graph(jfnk_batch* b, const float* u, const float* rhs, float* x, const std::vector<int>& act0,
                  const std::vector<double>& tol, const jfnk_gmres_opts& o, std::vector<int>& iters,
                  std::vector<int>& conv) {
    const int ni = b->ninst;
    const int max_iters = o.max_iters > 0 ? o.max_iters : o.m * o.max_restarts;
    hipStream_t s = b->stream;
    int rc;
    // start: activity and tolerances in, x = 0, frozen coefficients, ||u||, V_0 = rhs, beta
    for (int i = 0; i < ni; ++i) {
        b->hflags[i] = act0[i];
        b->htol[i] = tol[i];
    }
    JFNK_HIP(hipMemcpyAsync(b->d_active, b->hflags, ni * sizeof(int), hipMemcpyHostToDevice, s));
    JFNK_HIP(hipMemcpyAsync(b->d_tol, b->htol, ni * sizeof(double), hipMemcpyHostToDevice, s));
    {
        const BTab t = tab(b, 1, false), ta = tab(b, 1, true);
        hipLaunchKernelGGL((kb_zero<float>), dim3(b->nchunks), dim3(kB), 0, s, t, x);
        if (o.pc == JFNK_PC_PHYSICS)
            b_frozen_nu(b, ta, u);
        JFNK_HIP(hipGetLastError());
    }
    if ((rc = b_norm2<float>(b, u, b->scal + SB_UNORM2, S_STRIDE, FIN_STORE, true))) return rc;
    JFNK_HIP(hipMemcpyAsync(b->V32, rhs, b->ntot * sizeof(float), hipMemcpyDeviceToDevice, s));
    if ((rc = b_norm2<float>(b, b->V32, b->outv, 1, FIN_BETA, true))) return rc;
    const BDev d = bdev(b);
    hipLaunchKernelGGL(kb_dev_begin, dim3((ni + 255) / 256), dim3(256), 0, s, ni, d, (const double*)b->scal);
    JFNK_HIP(hipGetLastError());
    // the cycle graph, captured once per set of options
    const int key[8] = {o.m, o.sweeps, o.pc, o.ortho, max_iters, b->tune[3], b->tune[5], 1};
    if (!b->cycle_exec || !std::equal(key, key + 8, b->cyc_key)) {
        if (b->cycle_exec) {
            JFNK_HIP(hipGraphExecDestroy(b->cycle_exec));
            b->cycle_exec = nullptr;
        }
        JFNK_HIP(hipStreamSynchronize(s));
        hipGraph_t graph = nullptr;
        b->stream = b->cap_stream;
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = b_enqueue_cycle(b, u, rhs, x, o, max_iters);
            hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
            if (!rc && e2 != hipSuccess) e = e2;
        }
        b->stream = s;
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "capture of the ensemble cycle");
        e = hipGraphInstantiate(&b->cycle_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->cycle_exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        std::copy(key, key + 8, b->cyc_key);
    }
    while (true) {
        JFNK_HIP(hipGraphLaunch(b->cycle_exec, s));
        JFNK_HIP(hipStreamSynchronize(s));
        if (b->hdflags[1]) {
            set_error("non-finite Krylov norm in the batch");
            return JFNK_ERR_NONFINITE;
        }
        if (!b->hdflags[0]) break;
    }
    JFNK_HIP(hipMemcpyAsync(b->hres, b->d_iters, ni * sizeof(int), hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipMemcpyAsync(b->hres + ni, b->d_conv, ni * sizeof(int), hipMemcpyDeviceToHost, s));
    JFNK_HIP(hipStreamSynchronize(s));
    iters.assign(b->hres, b->hres + ni);
    conv.assign(b->hres + ni, b->hres + 2 * ni);
    return JFNK_OK;
}

// Lockstep flexible GMRES(m) in FP32 over the instances with act[i] = 1:
// J_i x_i = b_i to relative tolerance tol[i]; x of the others is left at zero.
int b_gmres(jfnk_batch* b, const float* u, const float* rhs, float* x, const std::vector<int>& act0,
            const std::vector<double>& tol, const jfnk_gmres_opts& o, std::vector<int>& iters,
            std::vector<int>& conv) {
    if (o.ortho == JFNK_ORTHO_ONE_REDUCTION && o.m < kDgMaxRows)
        return b_gmres_one_reduction(b, u, rhs, x, act0, tol, o, iters, conv);
    const int ni = b->ninst, m = o.m;
    const long long ntot = b->ntot;
    const int max_iters = o.max_iters > 0 ? o.max_iters : m * o.max_restarts;
    const double sqrt_eps = std::sqrt(1.1920928955078125e-07);
    hipStream_t s = b->stream;
    std::vector<int> act = act0;
    iters.assign(ni, 0);
    conv.assign(ni, 0);
    int rc;
    std::vector<double> bnorm, res;
    if ((rc = b_gmres_begin(b, u, rhs, x, o, act, conv, bnorm, res))) return rc;
    const BTab tall = tab(b, 1, false);
    while (true) {
        if (std::none_of(act.begin(), act.end(), [](int a) { return a; })) break;
        if ((rc = b_set_active(b, act))) return rc;
        const BTab ta = tab(b, 1, true);
        hipLaunchKernelGGL(kb_set_start, dim3((ni + 255) / 256), dim3(256), 0, s, ta, b->g, (const double*)b->scal, m);
        JFNK_HIP(hipGetLastError());
        std::vector<int> kcnt(ni, 0);
        std::vector<int> in_cycle = act;          // instances working in this cycle
        std::vector<int> cycle_done(ni, 0);
        for (int j = 0; j < m; ++j) {
            float* Vj = b->V32 + (long long)j * ntot;
            float* Vn = b->V32 + (long long)(j + 1) * ntot;
            float* Zj = b->Z32 + (long long)j * ntot;
            const int which = j == 0 ? SB_BETA : SB_WNORM;
            // z_j = M^-1 (V_j / norm)
            if (o.pc == JFNK_PC_PHYSICS) {
                float* bufs[2] = {Zj, b->t32};
                int cur = (o.sweeps % 2 == 0) ? 0 : 1;
                b_pc_diag(b, ta, Vj, (const double*)(b->scal + which), bufs[cur]);
                JFNK_HIP(hipGetLastError());
                for (int sw = 0; sw < o.sweeps; ++sw) {
                    JFNK_HIP(b_pc_sweep<float>(b, u, b->nu32, Vj, bufs[cur], bufs[1 - cur], b->tune[2 * 2 + 1]));
                    cur = 1 - cur;
                }
            } else {
                hipLaunchKernelGGL((kb_normalize_copy<float>), dim3(b->nchunks), dim3(kB), 0, s, ta, Vj,
                                   (const double*)b->scal, which, Zj);
                JFNK_HIP(hipGetLastError());
            }
            if ((rc = b_norm2<float>(b, Zj, b->scal + SB_VNORM2, S_STRIDE, FIN_EPS, true, sqrt_eps))) return rc;
            JFNK_HIP(b_jv<float>(b, u, Zj, b->scal + SB_EPS, Vn, b->tune[1 * 2 + 1]));
            if ((rc = b_cgs<float>(b, j + 1, CGS_DOT, nullptr, Vn, b->h1, j, m))) return rc;
            if ((rc = b_cgs<float>(b, j + 1, CGS_UPD_DOT, b->h1, Vn, b->h2, j, m))) return rc;
            if ((rc = b_cgs<float>(b, j + 1, CGS_UPD_NORM, b->h2, Vn, b->outv, j, m))) return rc;
            if ((rc = b_read_scal(b))) return rc;
            bool any = false;
            for (int i = 0; i < ni; ++i) {
                if (!act[i]) continue;
                const double wn = b->hscal[(long long)i * S_STRIDE + SB_WNORM];
                res[i] = b->hscal[(long long)i * S_STRIDE + SB_RES];
                if (!std::isfinite(wn) || !std::isfinite(res[i])) {
                    set_error("non-finite Krylov norm in the batch");
                    return JFNK_ERR_NONFINITE;
                }
                kcnt[i] = j + 1;
                iters[i]++;
                if (res[i] <= tol[i] * bnorm[i] || wn == 0.0 || iters[i] >= max_iters) {
                    act[i] = 0;
                    cycle_done[i] = 1;
                    conv[i] = res[i] <= tol[i] * bnorm[i] ? 1 : 0;
                } else {
                    any = true;
                }
            }
            if (!any) break;
            if ((rc = b_set_active(b, act))) return rc;
        }
        // solution update of every instance that worked in this cycle
        if ((rc = b_set_kcnt(b, kcnt))) return rc;
        hipLaunchKernelGGL(kb_backsolve, dim3((ni + 63) / 64), dim3(64), 0, s, tall, (const double*)b->H,
                           (const double*)b->g, (const int*)b->d_kcnt, m, b->y);
        JFNK_HIP(hipGetLastError());
        hipLaunchKernelGGL((kb_axpy_basis<float>), dim3(b->nchunks), dim3(kB), 0, s, tall, x, (const float*)b->Z32,
                           ntot, (const int*)b->d_kcnt, (const double*)b->y);
        JFNK_HIP(hipGetLastError());
        // instances still active restart from the true residual
        if (std::none_of(act.begin(), act.end(), [](int a) { return a; })) break;
        if ((rc = b_set_active(b, act))) return rc;
        if ((rc = b_restart_residual(b, u, rhs, x, act, conv))) return rc;
    }
    JFNK_HIP(hipStreamSynchronize(s));
    return JFNK_OK;
}

__global__ void k_background_batch(Geo g, jfnk_problem p, double* pbar, double* dpbar, double* sflux, float* pbar32,
                                   float* dpbar32, float* sflux32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < g.nz) {
        const double z = (t + 0.5) * g.dz;
        const double thb = p.theta0 + g.beta * z;
        const double pb = g.beta > 0.0 ? p.cp - (p.g / g.beta) * log1p(g.beta * z / p.theta0)
                                       : p.cp - p.g * z / p.theta0;
        pbar[t] = pb;
        dpbar[t] = -p.g / thb;
        pbar32[t] = (float)pb;
        dpbar32[t] = (float)(-p.g / thb);
    }
    if (t < g.nx * g.ny) {
        // the cell centre is rounded on its own, as the strip definition reads
        // (no multiply-add fused into the strip test)
#pragma clang fp contract(off)
        const double x = (t % g.nx + 0.5) * g.dx;
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
        const double q = H / (p.p_ref / (p.rgas * p.theta0) * p.cp) / g.dz;
        sflux[t] = q;
        sflux32[t] = (float)q;
    }
}

}  // namespace

extern "C" {

int jfnk_batch_destroy(jfnk_batch* b) {
    if (!b) return JFNK_OK;
    (void)hipStreamSynchronize(b->stream);
    void* ptrs[] = {b->d_geos, b->d_voff, b->d_poff, b->d_noff, b->d_tile_off[0], b->d_tile_off[1], b->d_tile_off[2],
                    b->d_tiles_x[0], b->d_tiles_x[1], b->d_tiles_x[2], b->d_pblk_off, b->d_eblk_off, b->d_chunk_off,
                    b->d_active, b->d_kcnt, b->V32, b->Z32, b->u32, b->b32, b->x32, b->t32, b->nu32, b->f64, b->R64,
                    b->bg64, b->bg32, b->H, b->Hraw, b->cs, b->sn, b->g, b->y, b->h1, b->h2, b->scal, b->outv,
                    b->partials, b->coef, b->d_incycle, b->d_conv, b->d_iters, b->d_dflags, b->d_tol, b->d_bnorm};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (b->hscal) (void)hipHostFree(b->hscal);
    if (b->hflags) (void)hipHostFree(b->hflags);
    if (b->hdflags) (void)hipHostFree(b->hdflags);
    if (b->htol) (void)hipHostFree(b->htol);
    if (b->hres) (void)hipHostFree(b->hres);
    if (b->cycle_exec) (void)hipGraphExecDestroy(b->cycle_exec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return JFNK_OK;
}

int jfnk_batch_create(const jfnk_problem* probs, int32_t ninst, int32_t max_m, void* stream, jfnk_batch** out) {
    if (!out || !probs || ninst < 1 || max_m < 1 || max_m + 1 > kMaxDots) {
        set_error("invalid argument to jfnk_batch_create");
        return JFNK_ERR_ARG;
    }
    *out = nullptr;
    jfnk_batch* b = new jfnk_batch();
    b->ninst = ninst;
    b->max_m = max_m;
    b->stream = (hipStream_t)stream;
    auto fail = [&](int code) {
        jfnk_batch_destroy(b);
        return code;
    };
    b->voff.push_back(0);
    b->poff.push_back(0);
    b->noff.push_back(0);
    for (int v = 0; v < 3; ++v) b->tile_off[v].push_back(0);
    b->pblk_off.push_back(0);
    b->eblk_off.push_back(0);
    b->chunk_off.push_back(0);
    long long nbg = 0;
    b->W = probs[0].dd_p == 3 ? 4 : 2;
    const int ew = 2 * b->W;    // ring-W extended grids: (nx + 2W) x (nz + 2W)
    for (int i = 0; i < ninst; ++i) {
        const jfnk_problem& p = probs[i];
        std::string why;
        if (p.dim != 2 || p.ny != 1 || p.nx < 8 || p.nz < 8 || !(p.dt > 0) || p.dd_p != probs[0].dd_p ||
            (p.dd_p != 2 && p.dd_p != 3) || p.closure < 0 ||
            p.closure > 3 || (p.closure == JFNK_CLOSURE_SMAGORINSKY && !(p.pr_t > 0)) ||
            (p.closure == JFNK_CLOSURE_DEARDORFF && (!(p.cs >= 0) || !(p.n_bv >= 0)))) {
            set_error("batch instance " + std::to_string(i) + ": unsupported or invalid problem (2D, nx and nz "
                      "at least 8, one dd_p of 2 or 3 for every instance)");
            return fail(JFNK_ERR_ARG);
        }
        b->probs.push_back(p);
        Geo g{};
        fill_geo(p, g);
        b->geos.push_back(g);
        const long long n = 4 * g.npts;
        b->voff.push_back(b->voff.back() + n);
        b->poff.push_back(b->poff.back() + g.npts);
        b->noff.push_back(b->noff.back() + (long long)(g.nx + ew) * (g.nz + ew));
        for (int v = 0; v < 3; ++v) {
            const int tz = tile_tz(v);
            const int tx = (g.nx + 63) / 64;
            b->tiles_x[v].push_back(tx);
            b->tile_off[v].push_back(b->tile_off[v].back() + tx * ((g.nz + tz - 1) / tz));
        }
        b->pblk_off.push_back(b->pblk_off.back() + (int)((g.npts + kB - 1) / kB));
        b->eblk_off.push_back(b->eblk_off.back() + (int)(((long long)(g.nx + ew) * (g.nz + ew) + kB - 1) / kB));
        b->chunk_off.push_back(b->chunk_off.back() + (int)((n + kChunk - 1) / kChunk));
        nbg += 2 * g.nz + g.nx;
    }
    b->ntot = b->voff.back();
    b->ptot = b->poff.back();
    b->netot = b->noff.back();
    b->nchunks = b->chunk_off.back();
    const long long ntot = b->ntot;
#define BALLOC(ptr, count)                                                   \
    do {                                                                     \
        hipError_t e_ = hipMalloc((void**)&(ptr), sizeof(*(ptr)) * (count)); \
        if (e_ != hipSuccess) {                                              \
            hip_fail(e_, "hipMalloc " #ptr);                                 \
            return fail(JFNK_ERR_HIP);                                       \
        }                                                                    \
    } while (0)
    BALLOC(b->d_geos, ninst);
    BALLOC(b->d_voff, ninst + 1);
    BALLOC(b->d_poff, ninst + 1);
    BALLOC(b->d_noff, ninst + 1);
    for (int v = 0; v < 3; ++v) {
        BALLOC(b->d_tile_off[v], ninst + 1);
        BALLOC(b->d_tiles_x[v], ninst);
    }
    BALLOC(b->d_pblk_off, ninst + 1);
    BALLOC(b->d_eblk_off, ninst + 1);
    BALLOC(b->d_chunk_off, ninst + 1);
    BALLOC(b->d_active, ninst);
    BALLOC(b->d_kcnt, ninst);
    BALLOC(b->V32, (size_t)(max_m + 1) * ntot);
    BALLOC(b->Z32, (size_t)max_m * ntot);
    BALLOC(b->u32, ntot);
    BALLOC(b->b32, ntot);
    BALLOC(b->x32, ntot);
    BALLOC(b->t32, ntot);
    BALLOC(b->nu32, b->netot);
    BALLOC(b->f64, ntot);
    BALLOC(b->R64, ntot);
    BALLOC(b->bg64, nbg);
    BALLOC(b->bg32, nbg);
    BALLOC(b->H, (size_t)ninst * (M + 1) * M);
    BALLOC(b->Hraw, (size_t)ninst * (M + 1) * M);
    BALLOC(b->cs, (size_t)ninst * M);
    BALLOC(b->sn, (size_t)ninst * M);
    BALLOC(b->g, (size_t)ninst * (M + 1));
    BALLOC(b->y, (size_t)ninst * M);
    BALLOC(b->h1, (size_t)ninst * M);
    BALLOC(b->h2, (size_t)ninst * M);
    BALLOC(b->scal, (size_t)ninst * S_STRIDE);
    BALLOC(b->outv, (size_t)ninst);
    BALLOC(b->partials, (size_t)b->nchunks * (kMaxDots + 2));   // the one-reduction pass uses 2 kDgMaxRows + 2
    BALLOC(b->coef, (size_t)ninst * kBdCoef);
    BALLOC(b->d_incycle, ninst);
    BALLOC(b->d_conv, ninst);
    BALLOC(b->d_iters, ninst);
    BALLOC(b->d_dflags, 2);
    BALLOC(b->d_tol, ninst);
    BALLOC(b->d_bnorm, ninst);
#undef BALLOC
    if (hipHostMalloc((void**)&b->hscal, (size_t)ninst * S_STRIDE * sizeof(double), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&b->hflags, (size_t)ninst * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->hdflags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->htol, (size_t)ninst * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->hres, (size_t)2 * ninst * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return fail(JFNK_ERR_HIP);
    }
    // background profiles and surface flux per instance
    long long o = 0;
    for (int i = 0; i < ninst; ++i) {
        Geo& g = b->geos[i];
        g.pbar64 = b->bg64 + o;
        g.dpbar64 = b->bg64 + o + g.nz;
        g.sflux64 = b->bg64 + o + 2 * g.nz;
        g.pbar32 = b->bg32 + o;
        g.dpbar32 = b->bg32 + o + g.nz;
        g.sflux32 = b->bg32 + o + 2 * g.nz;
        o += 2 * g.nz + g.nx;
        const int cnt = std::max(g.nz, g.nx);
        hipLaunchKernelGGL(k_background_batch, dim3((cnt + 255) / 256), dim3(256), 0, b->stream, g, b->probs[i],
                           (double*)g.pbar64, (double*)g.dpbar64, (double*)g.sflux64, (float*)g.pbar32,
                           (float*)g.dpbar32, (float*)g.sflux32);
        if (hipGetLastError() != hipSuccess) {
            set_error("background kernel launch failed");
            return fail(JFNK_ERR_HIP);
        }
    }
    auto up = [&](void* d, const void* h, size_t bytes) {
        return hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, b->stream) == hipSuccess;
    };
    bool ok = up(b->d_geos, b->geos.data(), ninst * sizeof(Geo)) && up(b->d_voff, b->voff.data(), (ninst + 1) * 8) &&
              up(b->d_poff, b->poff.data(), (ninst + 1) * 8) && up(b->d_noff, b->noff.data(), (ninst + 1) * 8) &&
              up(b->d_pblk_off, b->pblk_off.data(), (ninst + 1) * 4) &&
              up(b->d_eblk_off, b->eblk_off.data(), (ninst + 1) * 4) &&
              up(b->d_chunk_off, b->chunk_off.data(), (ninst + 1) * 4);
    for (int v = 0; v < 3 && ok; ++v)
        ok = up(b->d_tile_off[v], b->tile_off[v].data(), (ninst + 1) * 4) &&
             up(b->d_tiles_x[v], b->tiles_x[v].data(), ninst * 4);
    // per-instance constants in the scalar block: sqrt(N_i)
    std::vector<double> sc0((size_t)ninst * S_STRIDE, 0.0);
    for (int i = 0; i < ninst; ++i) sc0[(size_t)i * S_STRIDE + SB_SQRTN] = std::sqrt((double)(4 * b->geos[i].npts));
    ok = ok && up(b->scal, sc0.data(), sc0.size() * sizeof(double));
    if (!ok || hipStreamSynchronize(b->stream) != hipSuccess) {
        set_error("batch table upload failed");
        return fail(JFNK_ERR_HIP);
    }
    *out = b;
    return JFNK_OK;
}

int jfnk_batch_size(jfnk_batch* b, int64_t* total, int64_t* offsets) {
    if (!b) {
        set_error("null batch");
        return JFNK_ERR_ARG;
    }
    if (total) *total = b->ntot;
    if (offsets)
        for (int i = 0; i <= b->ninst; ++i) offsets[i] = b->voff[i];
    return JFNK_OK;
}

int jfnk_batch_apply_F(jfnk_batch* b, int32_t what, const double* u, const double* f, double* out) {
    if (!b || !u || !out || what < 0 || what > 2) {
        set_error("invalid argument to jfnk_batch_apply_F");
        return JFNK_ERR_ARG;
    }
    JFNK_HIP(b_apply_F<double>(b, u, f, out, what));
    return JFNK_OK;
}

int jfnk_batch_newton_step(jfnk_batch* b, const double* u_n, double* u, const jfnk_newton_opts* o,
                           jfnk_newton_info* infos, int32_t use_graph) {
    if (!b || !u_n || !u || !o || o->inner != JFNK_F32 || o->gm.m < 1 || o->gm.m > b->max_m ||
        (o->gm.pc != JFNK_PC_PHYSICS && o->gm.pc != JFNK_PC_NONE) || o->max_newton < 0 ||
        (o->gm.ortho != JFNK_ORTHO_CGS2 && o->gm.ortho != JFNK_ORTHO_ONE_REDUCTION)) {
        set_error("invalid argument to jfnk_batch_newton_step (FP32 inner solve, physics or no preconditioner, "
                  "a known Gram-Schmidt form)");
        return JFNK_ERR_ARG;
    }
    const int ni = b->ninst;
    const long long ntot = b->ntot;
    hipStream_t s = b->stream;
    int rc;
    JFNK_HIP(b_apply_F<double>(b, u_n, nullptr, b->f64, 1));
    // atol_i from ||u^n_i||
    if ((rc = b_norm2<double>(b, u_n, b->outv, 1, FIN_STORE, false))) return rc;
    std::vector<double> un2(ni);
    JFNK_HIP(hipMemcpyAsync(un2.data(), b->outv, ni * sizeof(double), hipMemcpyDeviceToHost, s));
    auto resid = [&](std::vector<double>& rn) -> int {
        JFNK_HIP(b_apply_F<double>(b, u, b->f64, b->R64, 2));
        int r2 = b_norm2<double>(b, b->R64, b->outv, 1, FIN_STORE, false);
        if (r2) return r2;
        JFNK_HIP(hipMemcpyAsync(rn.data(), b->outv, ni * sizeof(double), hipMemcpyDeviceToHost, s));
        JFNK_HIP(hipStreamSynchronize(s));
        for (auto& v : rn) v = std::sqrt(v);
        return JFNK_OK;
    };
    std::vector<double> rn(ni), r0(ni), tol(ni), rprev(ni), eta(ni, 0.5);
    if ((rc = resid(rn))) return rc;
    std::vector<int> act(ni), nit(ni, 0), gtot(ni, 0);
    for (int i = 0; i < ni; ++i) {
        r0[i] = rn[i];
        rprev[i] = rn[i];
        tol[i] = std::max(o->rtol * r0[i], o->atol_factor * (2.0 / b->probs[i].dt) * std::sqrt(un2[i]));
        act[i] = rn[i] > tol[i] ? 1 : 0;
    }
    for (int k = 0; k < o->max_newton; ++k) {
        for (int i = 0; i < ni; ++i)
            if (!std::isfinite(rn[i])) {
                set_error("non-finite Newton residual in batch instance " + std::to_string(i));
                return JFNK_ERR_NONFINITE;
            }
        if (std::none_of(act.begin(), act.end(), [](int a) { return a; })) break;
        std::vector<double> gt(ni, 0.0);
        for (int i = 0; i < ni; ++i) {
            if (!act[i]) continue;
            double e;
            if (o->forcing == 0) {
                if (nit[i] == 0) {
                    e = 0.5;
                } else {
                    e = 0.9 * std::pow(rn[i] / rprev[i], 2.0);
                    const double sg = 0.9 * eta[i] * eta[i];
                    if (sg > 0.1) e = std::max(e, sg);
                    e = std::min(e, 0.9);
                }
                e = std::min(std::max(e, 0.5 * tol[i] / rn[i]), 0.9);
            } else {
                e = o->eta;
            }
            eta[i] = std::max(e, o->eta_floor);
            gt[i] = eta[i];
        }
        JFNK_HIP(launch_cast<float, double>(b->u32, u, ntot, 1.0, s));
        JFNK_HIP(launch_cast<float, double>(b->b32, b->R64, ntot, -1.0, s));
        std::vector<int> gi, gc;
        rc = use_graph ? b_gmres_graph(b, b->u32, b->b32, b->x32, act, gt, o->gm, gi, gc)
                       : b_gmres(b, b->u32, b->b32, b->x32, act, gt, o->gm, gi, gc);
        if (rc) return rc;
        JFNK_HIP(launch_add_to64<float>(u, b->x32, ntot, s));     // x = 0 for finished instances
        for (int i = 0; i < ni; ++i)
            if (act[i]) {
                gtot[i] += gi[i];
                nit[i]++;
            }
        rprev = rn;
        if ((rc = resid(rn))) return rc;
        for (int i = 0; i < ni; ++i)
            if (act[i] && rn[i] <= tol[i]) act[i] = 0;
    }
    bool all = true;
    for (int i = 0; i < ni; ++i) {
        const bool c = rn[i] <= tol[i];
        all = all && c;
        if (infos) {
            infos[i].newton_iters = nit[i];
            infos[i].gmres_iters_total = gtot[i];
            infos[i].converged = c ? 1 : 0;
            infos[i].fallbacks = 0;
            infos[i].res0 = r0[i];
            infos[i].res_final = rn[i];
        }
    }
    return all ? JFNK_OK : JFNK_NOT_CONVERGED;
}

// Autotuner of the batched stencil stages (tile heights 4, 8, 16).
int jfnk_batch_tune(jfnk_batch* b, int32_t* tile_rows) {
    if (!b) {
        set_error("null batch");
        return JFNK_ERR_ARG;
    }
    hipStream_t s = b->stream;
    hipEvent_t e0, e1;
    JFNK_HIP(hipEventCreate(&e0));
    JFNK_HIP(hipEventCreate(&e1));
    std::vector<int> all(b->ninst, 1);
    int rc = b_set_active(b, all);
    if (rc) return rc;
    JFNK_HIP(hipMemsetAsync(b->V32, 0, 2 * b->ntot * sizeof(float), s));
    JFNK_HIP(hipMemsetAsync(b->f64, 0, b->ntot * sizeof(double), s));
    for (int stage = 0; stage < 3; ++stage) {
        float best = 1e30f;
        int bestv = 1;
        for (int var = 0; var < 3; ++var) {
            auto launch = [&]() -> hipError_t {
                if (stage == 0) return b_apply_F<double>(b, b->f64, nullptr, b->R64, 0, var);
                if (stage == 1) return b_jv<float>(b, b->V32, b->V32 + b->ntot, b->scal + SB_EPS, b->Z32, var);
                return b_pc_sweep<float>(b, b->V32, b->nu32, b->V32 + b->ntot, b->V32, b->Z32, var);
            };
            JFNK_HIP(launch());
            JFNK_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < 5; ++k) JFNK_HIP(launch());
            JFNK_HIP(hipEventRecord(e1, s));
            JFNK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            JFNK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestv = var;
            }
        }
        b->tune[stage * 2 + (stage == 0 ? 0 : 1)] = bestv;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (tile_rows) {
        tile_rows[0] = tile_tz(b->tune[0]);
        tile_rows[1] = tile_tz(b->tune[3]);
        tile_rows[2] = tile_tz(b->tune[5]);
    }
    return JFNK_OK;
}

}  // extern "C"
