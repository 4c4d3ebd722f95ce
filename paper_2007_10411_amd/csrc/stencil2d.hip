// Single-grid 2D stencil kernels: one workgroup per TX x TZ tile of the grid.
// The bodies live in stencil2d_impl.hpp; TZ is chosen per stage by the
// autotuner among the compiled variants 4, 8 and 16.

#include "stencil2d_impl.hpp"

namespace jfnk {

namespace {

using namespace s2d;

template <typename T, int TX, int TZ>
__global__ __launch_bounds__(256) void k_apply_F_2d(Geo g, const T* __restrict__ u, const T* __restrict__ f,
                                                    T* __restrict__ out, int what) {
    apply_F_tile<T, TX, TZ>(g, blockIdx.x * TX, blockIdx.y * TZ, u, f, out, what);
}

template <typename T>
__global__ __launch_bounds__(256) void k_frozen_nu_2d(Geo g, const T* __restrict__ u, T* __restrict__ nu) {
    frozen_nu_point<T>(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, u, nu);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pc_diag_2d(Geo g, const T* __restrict__ nu, T* __restrict__ vj,
                                                    const double* __restrict__ div, T* __restrict__ z,
                                                    EpsArgs ea) {
    __shared__ double red[4];
    const double acc = pc_diag_point<T>(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, nu, vj, div, z);
    if (ea.partials) partial_eps(ea, acc, red);
}

template <typename T, int TX, int TZ>
__global__ __launch_bounds__(256) void k_pc_sweep_2d(Geo g, const T* __restrict__ u, const T* __restrict__ nu,
                                                     const T* __restrict__ r, const T* __restrict__ zin,
                                                     T* __restrict__ zout, EpsArgs ea) {
    __shared__ double red[4];
    const double acc = pc_sweep_tile<T, TX, TZ>(g, blockIdx.x * TX, blockIdx.y * TZ, u, nu, r, zin, zout);
    if (ea.partials) partial_eps(ea, acc, red);
}

}  // namespace

// tile height variants (TX = 64); variant index v -> TZ = 4 << v
constexpr int kTX = 64;

inline dim3 tile_grid(const Geo& g, int tz) { return dim3((g.nx + kTX - 1) / kTX, (g.nz + tz - 1) / tz); }

#define JFNK_TZ_DISPATCH(var, KERNEL, T, grid_expr, ...)                                                   \
    do {                                                                                                   \
        if ((var) == 0)                                                                                    \
            hipLaunchKernelGGL((KERNEL<T, kTX, 4>), tile_grid(g, 4), dim3(256), 0, s, __VA_ARGS__);          \
        else if ((var) == 2)                                                                               \
            hipLaunchKernelGGL((KERNEL<T, kTX, 16>), tile_grid(g, 16), dim3(256), 0, s, __VA_ARGS__);        \
        else                                                                                               \
            hipLaunchKernelGGL((KERNEL<T, kTX, 8>), tile_grid(g, 8), dim3(256), 0, s, __VA_ARGS__);          \
    } while (0)

int tile_tz(int variant) { return variant == 0 ? 4 : (variant == 2 ? 16 : 8); }

template <typename T>
hipError_t launch_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, hipStream_t s, int var) {
    JFNK_TZ_DISPATCH(var, k_apply_F_2d, T, 0, g, u, f, out, what);
    return hipGetLastError();
}

// FP64 Jv tiles of height 16 would need 165 KB of LDS (above the 160 KB of a CU)
template <typename T, int TX, int TZ>
__global__ __launch_bounds__(256) void k_jv_2d(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                      double eps_in, const double* __restrict__ eps_dev,
                                                      T* __restrict__ out) {
    constexpr int TZC = (sizeof(T) == 8 && TZ > 8) ? 8 : TZ;
    jv_tile<T, TX, TZC>(g, blockIdx.x * TX, blockIdx.y * TZC, u, v, eps_in, eps_dev, out);
}

template <typename T>
hipError_t launch_jv(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, T* jv,
                     hipStream_t s, int var) {
    if (sizeof(T) == 8 && var == 2) var = 1;
    JFNK_TZ_DISPATCH(var, k_jv_2d, T, 0, g, u, v, eps, eps_dev, jv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_frozen_nu(const Geo& g, const T* u, T* nu, hipStream_t s) {
    const long long ne = (long long)(g.nx + 4) * (g.nz + 4);
    const int nb = (int)((ne + 255) / 256);
    hipLaunchKernelGGL((k_frozen_nu_2d<T>), dim3(nb), dim3(256), 0, s, g, u, nu);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pc_diag(const Geo& g, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea,
                          hipStream_t s) {
    const int nb = (int)((g.npts + 255) / 256);
    hipLaunchKernelGGL((k_pc_diag_2d<T>), dim3(nb), dim3(256), 0, s, g, nu, vj, div, z, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    return launch_eps_finish(nb, ea, s);
}

template <typename T>
hipError_t launch_pc_sweep(const Geo& g, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                           const EpsArgs& ea, hipStream_t s, int var) {
    JFNK_TZ_DISPATCH(var, k_pc_sweep_2d, T, 0, g, u, nu, r, zin, zout, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    const dim3 grid = tile_grid(g, tile_tz(var));
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
