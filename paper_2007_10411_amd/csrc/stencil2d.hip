// Single-grid 2D stencil kernels.  Tiles: one workgroup per TX x TZ tile of the
// grid, bodies in stencil2d_impl.hpp, TZ 4, 8 or 16.  Row marching (residual and
// Jv): one workgroup per 64-column strip walking down 32, 64 or 256 rows.  The
// autotuner picks the shape per stage and precision.

#include "stencil2d_impl.hpp"

namespace jfnk {

namespace {

using namespace s2d;

// Tile heights that fit in LDS for each stencil half-width W (the launchers use
// the same caps for their grids): FP64 Jv tiles stop at 8 rows (4 for W = 4),
// FP64 preconditioner sweeps at 8 rows for W = 4.
template <typename T, int TZ, int W> constexpr int jv_tz() {
    return sizeof(T) == 8 ? (W == 4 ? 4 : (TZ > 8 ? 8 : TZ)) : TZ;
}
template <typename T, int TZ, int W> constexpr int sweep_tz() {
    return (sizeof(T) == 8 && W == 4 && TZ > 8) ? 8 : TZ;
}

template <typename T, int TX, int TZ, int W>
__global__ __launch_bounds__(256) void k_apply_F_2d(Geo g, const T* __restrict__ u, const T* __restrict__ f,
                                                    T* __restrict__ out, int what) {
    apply_F_tile<T, TX, TZ, W>(g, blockIdx.x * TX, blockIdx.y * TZ, u, f, out, what);
}

template <typename T, int W>
__global__ __launch_bounds__(256) void k_frozen_nu_2d(Geo g, const T* __restrict__ u, T* __restrict__ nu) {
    frozen_nu_point<T, W>(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, u, nu);
}

template <typename T, int W>
__global__ __launch_bounds__(256) void k_pc_diag_2d(Geo g, const T* __restrict__ nu, T* __restrict__ vj,
                                                    const double* __restrict__ div, T* __restrict__ z,
                                                    EpsArgs ea) {
    __shared__ double red[4];
    const double acc = pc_diag_point<T, W>(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, nu, vj, div, z);
    if (ea.partials) partial_eps(ea, acc, red);
}

template <typename T, int TX, int TZ, int W>
__global__ __launch_bounds__(256) void k_pc_sweep_2d(Geo g, const T* __restrict__ u, const T* __restrict__ nu,
                                                     const T* __restrict__ r, const T* __restrict__ zin,
                                                     T* __restrict__ zout, EpsArgs ea) {
    __shared__ double red[4];
    constexpr int TZC = sweep_tz<T, TZ, W>();
    const double acc = pc_sweep_tile<T, TX, TZC, W>(g, blockIdx.x * TX, blockIdx.y * TZC, u, nu, r, zin, zout);
    if (ea.partials) partial_eps(ea, acc, red);
}

// ---------------------------------------------------------------------------
// Row-marching residual and Jv.  A workgroup owns a strip of MX columns and
// walks down a chunk of zc rows, RB rows per step.  Primitive rows (halo 2W
// in x) live in a ring of RB + 3W LDS rows, the stress and heat flux of the
// rows in a ring of RB + 2W, so each row is fetched from HBM once per chunk
// (the tile kernels fetch the 2W-row halo of every tile again).  The next
// step's rows are loaded to registers while the current step computes.
//
// Strip shape: a step derives RB rows of MX + 2W columns and finishes RB rows
// of MX columns on 256 threads.  MX + 2W = 128 with RB = 2, or 64 with RB = 4,
// is one derived point per thread (64 columns would leave 4 (64 + 2W) points
// per step, a second pass for 8 W of them).
// ---------------------------------------------------------------------------
// FP32 with W = 2: 124 x 2 (LDS 49 KB, three workgroups per CU).  Otherwise
// (64 - 2W) x 4: the wide strip's LDS (95 KB for FP32 with W = 4, twice that in
// FP64) would leave one workgroup per CU.
template <typename T, int W> struct MarchShape {
    static constexpr bool kWide = sizeof(T) == 4 && W == 2;
    static constexpr int MX = kWide ? 128 - 2 * W : 64 - 2 * W, RB = kWide ? 2 : 4;
};

// One group of RB primitive rows of NF fields (fields 4.. from the second
// state), columns x0 - 2W .. x0 + MX + 2W - 1: fixed positions per thread, so
// the reflected source columns and their x-parity signs are set once.
template <typename T, int W, int NF, int MX, int RB>
struct RowStage {
    static constexpr int SX = MX + 4 * W, N = RB * SX;
    static constexpr int POS = (N + 255) / 256;
    int col[POS];
    int lrow[POS];
    unsigned xneg[POS];
    unsigned neg[POS];
    T r[POS][NF];
    __device__ __forceinline__ void init(const Geo& g, int x0) {
#pragma unroll
        for (int p = 0; p < POS; ++p) {
            const int idx = min((int)threadIdx.x + p * 256, N - 1);
            const int lr = idx / SX, lx = idx - lr * SX;
            int sx;
            col[p] = map_axis(x0 + lx - 2 * W, g.nx, g.bcl == JFNK_BC_PERIODIC, sx);
            lrow[p] = lr;
            unsigned m = 0u;
#pragma unroll
            for (int f = 0; f < NF; ++f)
                if (sign2d(f & 3, sx, 0, g.bcv) < 0) m |= 1u << f;
            xneg[p] = m;
        }
    }
    // rows rbase .. rbase + RB - 1 (reflected at the walls)
    __device__ __forceinline__ void load(const Geo& g, const T* __restrict__ a, const T* __restrict__ b, int rbase) {
        const long long np = g.npts;
#pragma unroll
        for (int p = 0; p < POS; ++p) {
            int sz;
            const int row = map_axis(rbase + lrow[p], g.nz, g.bcv == JFNK_BC_PERIODIC, sz);
            const long long off = (long long)row * g.nx + col[p];
            unsigned m = xneg[p];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                r[p][f] = (f < 4 ? a : b)[(long long)(f & 3) * np + off];
                if (sign2d(f & 3, 0, sz, g.bcv) < 0) m ^= 1u << f;
            }
            neg[p] = m;
        }
    }
    // into ring [f][NA][SX]; slot0 is the ring slot of row rbase.  With two
    // states (NF = 8) the first four fields go in as u + e v.
    template <int NA>
    __device__ __forceinline__ void store(T* dst, int slot0, T e) const {
#pragma unroll
        for (int p = 0; p < POS; ++p) {
            const int idx = (int)threadIdx.x + p * 256;
            if (idx < N) {
                const int lx = idx - lrow[p] * SX;
                T* d = dst + ((slot0 + lrow[p]) % NA) * SX + lx;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T v = (NF == 8 && f < 4) ? r[p][f] + e * r[p][f + 4] : r[p][f];
                    d[f * NA * SX] = (neg[p] >> f) & 1u ? -v : v;
                }
            }
        }
    }
};

template <typename T, int W, bool JV>
__global__ __launch_bounds__(256) void k_march_2d(Geo g, int zc, const T* __restrict__ u, const T* __restrict__ v,
                                                  double eps_in, const double* __restrict__ eps_dev,
                                                  const T* __restrict__ f, T* __restrict__ out, int what) {
    constexpr int MX = MarchShape<T, W>::MX, RB = MarchShape<T, W>::RB;
    constexpr int H = 2 * W, SX = MX + 2 * H, DX = MX + 2 * W;
    constexpr int NF = JV ? 8 : 4;
    // ring rows: RB + 3W in the march, 4W for the prologue's derived rows
    constexpr int NA = RB + 3 * W > 4 * W ? RB + 3 * W : 4 * W, NB = RB + 2 * W;
    constexpr int AFS = NA * SX, BFS = NB * DX;   // field strides of the rings
    constexpr int PW = (MX + 63) / 64 * 64;       // threads per output row
    static_assert(RB * PW <= 256 && H % RB == 0, "a step's rows fit the workgroup");
    __shared__ T sa[NF * AFS];
    __shared__ T sd[5 * BFS];
    const int tid = threadIdx.x;
    // Workgroups go round-robin to the 8 XCDs; give each XCD a contiguous run of
    // the strip-fastest order so that neighbouring strips, which share their
    // halo cache lines, run at the same time under the same L2.
    int bx, by;
    {
        const int nb = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x;
        const int q = nb / 8, r = nb % 8, xcd = lin % 8, k = lin / 8;
        const int logical = xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
        bx = logical % gridDim.x;
        by = logical / gridDim.x;
    }
    const int x0 = bx * MX, z0 = by * zc, z1 = min(z0 + zc, g.nz);
    const int ra0 = z0 - H;   // primitive row in ring slot 0
    const int rd0 = z0 - W;   // derived row in ring slot 0
    const T ihx = T(g.idx), ihz = T(g.idz);
    const T e = JV ? T(eps_dev ? *eps_dev : eps_in) : T(0);
    auto slotA = [&](int r) { return (r - ra0) % NA; };
    auto slotD = [&](int d) { return (d - rd0) % NB; };
    // ring pointers of 2W + 1 consecutive rows from the slot of the first
    auto rows = [](const T* base, int s, int stride, int n_slots, const T** r) {
#pragma unroll
        for (int k = 0; k <= 2 * W; ++k) {
            r[k] = base + s * stride;
            s = s + 1 == n_slots ? 0 : s + 1;
        }
    };
    auto prim = [&](int row, int c) {   // accessor of the primitives at (row, LDS column c)
        RingAcc<T, AFS, W> P;
        rows(sa + c, slotA(row - W), SX, NA, P.r);
        return P;
    };
    // stress and heat flux (or their differences) of derived rows d0 .. d0 + nrows - 1
    auto derive = [&](int d0, int nrows) {
        for (int idx = tid; idx < nrows * DX; idx += 256) {
            const int lr = idx / DX, lx = idx - lr * DX;
            const int d = d0 + lr;
            const RingAcc<T, AFS, W> PA = prim(d, lx + W);
            T dd[5];
            if constexpr (JV) {
                RingAcc<T, AFS, W> PB;
#pragma unroll
                for (int k = 0; k <= 2 * W; ++k) PB.r[k] = PA.r[k] + 4 * AFS;
                derived_jv_pt<W>(g, PA, PB, e, ihx, ihz, dd);
            } else {
                derived_F_pt<W>(g, PA, ihx, ihz, dd);
            }
            T* o = sd + slotD(d) * DX + lx;
#pragma unroll
            for (int k = 0; k < 5; ++k) o[k * BFS] = dd[k];
        }
    };

    RowStage<T, W, NF, MX, RB> st;
    st.init(g, x0);
    // prologue: primitive rows z0 - 2W .. z0 + 2W - 1, derived rows z0 - W .. z0 + W - 1
    for (int rb = z0 - H; rb < z0 + H; rb += RB) {
        st.load(g, u, v, rb);
        st.template store<NA>(sa, slotA(rb), e);
    }
    __syncthreads();
    derive(z0 - W, 2 * W);
    __syncthreads();
    const int nsteps = (z1 - z0 + RB - 1) / RB;
    st.load(g, u, v, z0 + H);
    const int ty = tid / PW, tx = tid - ty * PW;
    const bool owner = ty < RB && tx < MX;
    for (int k = 0; k < nsteps; ++k) {
        const int rb = z0 + k * RB;
        st.template store<NA>(sa, slotA(rb + H), e);
        __syncthreads();
        if (k + 1 < nsteps) st.load(g, u, v, rb + RB + H);
        derive(rb + W, RB);
        __syncthreads();
        const int gz = rb + ty, gx = x0 + tx;
        if (owner && gz < z1 && gx < g.nx) {
            const RingAcc<T, AFS, W> PA = prim(gz, tx + H);
            RingAcc<T, BFS, W> D;
            rows(sd + tx + W, slotD(gz - W), DX, NB, D.r);
            if constexpr (JV) {
                RingAcc<T, AFS, W> PB;
#pragma unroll
                for (int q = 0; q <= 2 * W; ++q) PB.r[q] = PA.r[q] + 4 * AFS;
                T o[4];
                point_jv_pt<W>(g, PA, PB, D, gz, e, ihx, ihz, o);
                const long long np = g.npts, off = (long long)gz * g.nx + gx;
#pragma unroll
                for (int q = 0; q < 4; ++q) out[q * np + off] = o[q];
            } else {
                T Fv[4];
                point_F_pt<W>(g, PA, D, gz, ihx, ihz, Fv);
                const T uv[4] = {PA.at(0, 0, 0), PA.at(1, 0, 0), PA.at(2, 0, 0), PA.at(3, 0, 0)};
                write_F(g, f, out, gz, gx, uv, Fv, what);
            }
        }
        __syncthreads();
    }
}

// rows per marching workgroup of variants 3, 4, 5
inline int march_rows(int var) { return var == 3 ? 32 : (var == 4 ? 64 : 256); }

template <typename T, bool JV>
hipError_t launch_march(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, const T* f, T* out,
                        int what, hipStream_t s, int var) {
    const int zc = march_rows(var);
    const int mx = g.W == 4 ? MarchShape<T, 4>::MX : MarchShape<T, 2>::MX;
    const dim3 grid((g.nx + mx - 1) / mx, (g.nz + zc - 1) / zc);
    if (g.W == 4)
        hipLaunchKernelGGL((k_march_2d<T, 4, JV>), grid, dim3(256), 0, s, g, zc, u, v, eps, eps_dev, f, out, what);
    else
        hipLaunchKernelGGL((k_march_2d<T, 2, JV>), grid, dim3(256), 0, s, g, zc, u, v, eps, eps_dev, f, out, what);
    return hipGetLastError();
}

}  // namespace

// tile height variants (TX = 64); variant index v -> TZ = 4 << v
constexpr int kTX = 64;

inline dim3 tile_grid(const Geo& g, int tz) { return dim3((g.nx + kTX - 1) / kTX, (g.nz + tz - 1) / tz); }

// TZ variant x stencil half-width W (g.W); CAP(TZ) is the tile height the
// kernel really uses (its grid)
#define JFNK_TZ_DISPATCH(var, KERNEL, T, CAP, ...)                                                         \
    do {                                                                                                   \
        if (g.W == 4) {                                                                                    \
            if ((var) == 0)                                                                                \
                hipLaunchKernelGGL((KERNEL<T, kTX, 4, 4>), tile_grid(g, CAP(4, 4)), dim3(256), 0, s, __VA_ARGS__);   \
            else if ((var) == 2)                                                                           \
                hipLaunchKernelGGL((KERNEL<T, kTX, 16, 4>), tile_grid(g, CAP(16, 4)), dim3(256), 0, s, __VA_ARGS__); \
            else                                                                                           \
                hipLaunchKernelGGL((KERNEL<T, kTX, 8, 4>), tile_grid(g, CAP(8, 4)), dim3(256), 0, s, __VA_ARGS__);   \
        } else {                                                                                           \
            if ((var) == 0)                                                                                \
                hipLaunchKernelGGL((KERNEL<T, kTX, 4, 2>), tile_grid(g, CAP(4, 2)), dim3(256), 0, s, __VA_ARGS__);   \
            else if ((var) == 2)                                                                           \
                hipLaunchKernelGGL((KERNEL<T, kTX, 16, 2>), tile_grid(g, CAP(16, 2)), dim3(256), 0, s, __VA_ARGS__); \
            else                                                                                           \
                hipLaunchKernelGGL((KERNEL<T, kTX, 8, 2>), tile_grid(g, CAP(8, 2)), dim3(256), 0, s, __VA_ARGS__);   \
        }                                                                                                  \
    } while (0)
#define JFNK_NO_CAP(tz, w) (tz)

int tile_tz(int variant) {
    if (variant >= 3) return march_rows(variant);
    return variant == 0 ? 4 : (variant == 2 ? 16 : 8);
}

template <typename T>
hipError_t launch_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, hipStream_t s, int var) {
    if (var >= 3) return launch_march<T, false>(g, u, nullptr, 0.0, nullptr, f, out, what, s, var);
    JFNK_TZ_DISPATCH(var, k_apply_F_2d, T, JFNK_NO_CAP, g, u, f, out, what);
    return hipGetLastError();
}

// FP64 Jv tiles of height 16 would need 165 KB of LDS (above the 160 KB of a CU)
template <typename T, int TX, int TZ, int W>
__global__ __launch_bounds__(256) void k_jv_2d(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                      double eps_in, const double* __restrict__ eps_dev,
                                                      T* __restrict__ out) {
    constexpr int TZC = jv_tz<T, TZ, W>();
    jv_tile<T, TX, TZC, W>(g, blockIdx.x * TX, blockIdx.y * TZC, u, v, eps_in, eps_dev, out);
}

template <typename T>
hipError_t launch_jv(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, T* jv,
                     hipStream_t s, int var) {
    if (var >= 3) return launch_march<T, true>(g, u, v, eps, eps_dev, nullptr, jv, 0, s, var);
#define JFNK_JV_CAP(tz, w) ((w) == 4 ? jv_tz<T, tz, 4>() : jv_tz<T, tz, 2>())
    JFNK_TZ_DISPATCH(var, k_jv_2d, T, JFNK_JV_CAP, g, u, v, eps, eps_dev, jv);
#undef JFNK_JV_CAP
    return hipGetLastError();
}

template <typename T>
hipError_t launch_frozen_nu(const Geo& g, const T* u, T* nu, hipStream_t s) {
    const long long ne = (long long)(g.nx + 2 * g.W) * (g.nz + 2 * g.W);
    const int nb = (int)((ne + 255) / 256);
    if (g.W == 4)
        hipLaunchKernelGGL((k_frozen_nu_2d<T, 4>), dim3(nb), dim3(256), 0, s, g, u, nu);
    else
        hipLaunchKernelGGL((k_frozen_nu_2d<T, 2>), dim3(nb), dim3(256), 0, s, g, u, nu);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pc_diag(const Geo& g, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea,
                          hipStream_t s) {
    const int nb = (int)((g.npts + 255) / 256);
    if (g.W == 4)
        hipLaunchKernelGGL((k_pc_diag_2d<T, 4>), dim3(nb), dim3(256), 0, s, g, nu, vj, div, z, ea);
    else
        hipLaunchKernelGGL((k_pc_diag_2d<T, 2>), dim3(nb), dim3(256), 0, s, g, nu, vj, div, z, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    return launch_eps_finish(nb, ea, s);
}

template <typename T>
hipError_t launch_pc_sweep(const Geo& g, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                           const EpsArgs& ea, hipStream_t s, int var) {
#define JFNK_SWEEP_CAP(tz, w) ((w) == 4 ? sweep_tz<T, tz, 4>() : sweep_tz<T, tz, 2>())
    JFNK_TZ_DISPATCH(var, k_pc_sweep_2d, T, JFNK_SWEEP_CAP, g, u, nu, r, zin, zout, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    const int tz = tile_tz(var);
    const dim3 grid = tile_grid(g, g.W == 4 ? (tz == 4 ? JFNK_SWEEP_CAP(4, 4) : tz == 16 ? JFNK_SWEEP_CAP(16, 4)
                                                                                         : JFNK_SWEEP_CAP(8, 4))
                                            : tz);
#undef JFNK_SWEEP_CAP
    return launch_eps_finish((int)(grid.x * grid.y), ea, s);
}

#define JFNK_INST(T)                                                                                          \
    template hipError_t launch_apply_F<T>(const Geo&, const T*, const T*, T*, int, hipStream_t, int);          \
    template hipError_t launch_jv<T>(const Geo&, const T*, const T*, double, const double*, T*, hipStream_t,   \
                                     int);                                                                     \
    template hipError_t launch_frozen_nu<T>(const Geo&, const T*, T*, hipStream_t);                            \
    template hipError_t launch_pc_diag<T>(const Geo&, const T*, T*, const double*, T*, const EpsArgs&,         \
                                          hipStream_t);                                                        \
    template hipError_t launch_pc_sweep<T>(const Geo&, const T*, const T*, const T*, const T*, T*,              \
                                           const EpsArgs&, hipStream_t, int);
JFNK_INST(double)
JFNK_INST(float)
#undef JFNK_INST

}  // namespace jfnk
