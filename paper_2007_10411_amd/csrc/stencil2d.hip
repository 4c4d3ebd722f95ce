// Single-grid 2D stencil kernels: one workgroup per TX x TZ tile of the grid.
// The bodies live in stencil2d_impl.hpp; TZ is chosen per stage by the
// autotuner among the compiled variants 4, 8 and 16.

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

int tile_tz(int variant) { return variant == 0 ? 4 : (variant == 2 ? 16 : 8); }

template <typename T>
hipError_t launch_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, hipStream_t s, int var) {
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
