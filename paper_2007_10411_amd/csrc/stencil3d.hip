// 3D stencil kernels of the JFNK hot path (gfx950).  Same discretisation as the
// 2D kernels (sections 2.1-2.4, equations 1-5 and 9): 5-point DD derivative,
// skew-symmetric convection, Smagorinsky stress, mirror-parity ghosts.  Fields
// (u, v, w, p', theta').
//
// The composite stencil D(tau(D u)) reaches 4 points along each axis and 2 x 2
// across axes, so each operator runs as two passes:
//   pass 1  the stress tau (6 components) and heat flux q (3) -- or their
//           finite-difference differences for Jv -- on the grid extended by a
//           ring of 2, written to an HBM buffer [9][nz+4][ny+4][nx+4];
//   pass 2  per grid point: convection, pressure gradient, divergence, buoyancy
//           and the divergences of tau and q.
// Both passes march along z through LDS windows of 5 planes (k3m_*), and so
// does the Jacobi sweep of the preconditioner (k3m_pc_sweep); the frozen
// viscosity and the diagonal start run one thread per point, x fastest.

#include <algorithm>

#include "jfnk_internal.hpp"
#include "reduce.hpp"
#include "exchange.hpp"

namespace jfnk {

namespace {

__device__ __forceinline__ int map3(int e, int n, bool periodic, int& side) {
    side = 0;
    if (periodic) {
        int r = e < 0 ? e + n : (e >= n ? e - n : e);
        if (r < 0 || r >= n) {
            r = e % n;
            r = r < 0 ? r + n : r;
        }
        return r;
    }
    if (e < 0) {
        side = 1;
        e = -1 - e;
    } else if (e >= n) {
        side = 2;
        e = 2 * n - 1 - e;
    }
    return e < 0 ? 0 : (e >= n ? n - 1 : e);
}

// Reflection sign of 3D field f (0 u, 1 v, 2 w, 3 p, 4 theta).
__device__ __forceinline__ bool odd3(int f, int sx, int sy, int sz, int bcv) {
    bool o = false;
    if (sx && f == 0) o = !o;
    if (sy && f == 1) o = !o;
    if (sz) {
        if (f == 2) o = !o;
        else if ((f == 0 || f == 1) && bcv == JFNK_BC_NO_SLIP_BOTTOM && sz == 1) o = !o;
    }
    return o;
}

template <typename T>
__device__ __forceinline__ T d5(T m2, T m1, T p1, T p2, T ih) {
    // weights scaled by 1/h once (shared by every derivative along the axis)
    return (T(2.0 / 3.0) * ih) * (p1 - m1) - (T(1.0 / 12.0) * ih) * (p2 - m2);
}

// field f of a state at (possibly ghost) position (x, y, z)
template <typename T>
__device__ __forceinline__ T ld(const Geo& g, const T* __restrict__ u, int f, int x, int y, int z) {
    int sx, sy, sz;
    const bool lat = g.bcl == JFNK_BC_PERIODIC;
    const int mx = map3(x, g.nx, lat, sx), my = map3(y, g.ny, lat, sy);
    const int mz = map3(z, g.nz, g.bcv == JFNK_BC_PERIODIC, sz);
    const T v = u[(long long)f * g.npts + ((long long)mz * g.ny + my) * g.nx + mx];
    return odd3(f, sx, sy, sz, g.bcv) ? -v : v;
}

// derivative of field f along axis a (0 x, 1 y, 2 z) at (x, y, z)
template <typename T>
__device__ __forceinline__ T dfield(const Geo& g, const T* __restrict__ u, int f, int a, int x, int y, int z) {
    const int ex = a == 0, ey = a == 1, ez = a == 2;
    const T ih = T(a == 0 ? g.idx : (a == 1 ? g.idy : g.idz));
    return d5(ld(g, u, f, x - 2 * ex, y - 2 * ey, z - 2 * ez), ld(g, u, f, x - ex, y - ey, z - ez),
              ld(g, u, f, x + ex, y + ey, z + ez), ld(g, u, f, x + 2 * ex, y + 2 * ey, z + 2 * ez), ih);
}

// extended-buffer access: component c at grid position (x, y, z), |offset| <= 2
template <typename T>
__device__ __forceinline__ T ldx(const Geo& g, const T* __restrict__ d, int c, int x, int y, int z) {
    const long long ex = g.nx + 4, ey = g.ny + 4, ez = g.nz + 4;
    return d[(long long)c * ex * ey * ez + ((long long)(z + 2) * ey + (y + 2)) * ex + (x + 2)];
}

template <typename T>
__device__ __forceinline__ T dext(const Geo& g, const T* __restrict__ d, int c, int a, int x, int y, int z) {
    const int ex = a == 0, ey = a == 1, ez = a == 2;
    const T ih = T(a == 0 ? g.idx : (a == 1 ? g.idy : g.idz));
    return d5(ldx(g, d, c, x - 2 * ex, y - 2 * ey, z - 2 * ez), ldx(g, d, c, x - ex, y - ey, z - ez),
              ldx(g, d, c, x + ex, y + ey, z + ez), ldx(g, d, c, x + 2 * ex, y + 2 * ey, z + 2 * ez), ih);
}

// Isotropic (nu, K_theta) of S:S = s2; for the anisotropic closure nu is the
// Smagorinsky viscosity from which its coefficients derive.
template <typename T>
__device__ __forceinline__ void closure3(const Geo& g, T s2, T& nu, T& kth) {
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
        nu = T(g.smag) * sqrt(T(2) * s2);
        kth = nu * T(g.inv_pr);
    } else if (g.closure == JFNK_CLOSURE_CONST_K) {
        nu = T(g.k_m);
        kth = T(g.k_h);
    } else {
        nu = T(0);
        kth = T(0);
    }
}

// symmetric strain (xx, yy, zz, xy, xz, yz) of the velocity of a state
template <typename T>
__device__ __forceinline__ void strain3(const Geo& g, const T* __restrict__ u, int x, int y, int z, T S[6],
                                        T th[3]) {
    T gr[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] = dfield(g, u, i, j, x, y, z);
    S[0] = gr[0][0];
    S[1] = gr[1][1];
    S[2] = gr[2][2];
    S[3] = T(0.5) * (gr[0][1] + gr[1][0]);
    S[4] = T(0.5) * (gr[0][2] + gr[2][0]);
    S[5] = T(0.5) * (gr[1][2] + gr[2][1]);
#pragma unroll
    for (int j = 0; j < 3; ++j) th[j] = dfield(g, u, 4, j, x, y, z);
}

template <typename T>
__device__ __forceinline__ T frob3(const T a[6], const T b[6]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + T(2) * (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]);
}

// exchange coefficients (horizontal, vertical) of S:S = s2
template <typename T>
__device__ __forceinline__ Coef<T> closure3c(const Geo& g, T s2) {
    if (g.closure == JFNK_CLOSURE_DEARDORFF) return deardorff_coef(g, T(sqrt(s2)));
    T nu, kth;
    closure3(g, s2, nu, kth);
    return {nu, nu, kth, kth};
}

// stress components xx, yy, zz, xy, xz, yz: the ones with a z index take the
// vertical coefficient
__device__ __forceinline__ bool vert3(int comp) { return comp == 2 || comp == 4 || comp == 5; }

__device__ __forceinline__ bool ext_point(const Geo& g, long long i, int& x, int& y, int& z) {
    const long long ex = g.nx + 4, ey = g.ny + 4, ez = g.nz + 4;
    if (i >= ex * ey * ez) return false;
    x = (int)(i % ex) - 2;
    y = (int)((i / ex) % ey) - 2;
    z = (int)(i / (ex * ey)) - 2;
    return true;
}

// stress component index of (i, j)
__device__ __forceinline__ int tix(int i, int j) {
    if (i == j) return i;
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

// ---------------------------------------------------------------------------
// z-marching operator kernels.  A workgroup owns a TX x TY column of points and
// walks through a chunk of kZC planes; a ring of 5 planes of the staged fields
// (the tile grown by 2 in x and y, reflected ghosts included) lives in LDS, so
// every neighbour along x, y and z of the 5-point derivative is an LDS read and
// every state value is fetched from HBM once per workgroup (plus the x-y halo).
// ---------------------------------------------------------------------------
constexpr int kMTX = 32;       // points per workgroup along x
constexpr int kZC = 16;        // planes per workgroup

template <int TY, int H = 2> struct MarchGeom {   // window region: the columns grown by H
    static constexpr int SX = kMTX + 2 * H, SY = TY + 2 * H, P = SX * SY;
};

// Register-staged copy of one plane of NF fields over the window region whose
// (0, 0) is grid point (xa, ya).  Each thread owns fixed in-plane positions of
// the region (idx = threadIdx.x + p NTHR), so their reflected source offsets and
// the x/y parity signs are computed once (init); per plane only the z mapping
// changes.  load() issues every global load of a plane, store() writes it to
// LDS as [field][position]; issued one plane ahead, the loads run under the
// compute of the current plane.  Fields 0..NS-1 come from state a, NS..2NS-1
// from state b; with SKIP_P the pressure is left out (field k is state field
// k < 3 ? k : 4).
template <typename T, int NF, int TY, int NTHR, int NS, bool SKIP_P, int H = 2>
struct Stager {
    using MG = MarchGeom<TY, H>;
    static constexpr int POS = (MG::P + NTHR - 1) / NTHR;
    static_assert(NF <= 32, "sign bits");
    int off[POS];          // in-plane source index (0 for positions past the region)
    unsigned xyneg[POS];   // fields negated by the x/y reflection
    unsigned zneg;         // fields negated by the z reflection of the loaded plane
    T r[POS][NF];
    __device__ __forceinline__ static int sfield(int f) {
        const int k = f < NS ? f : f - NS;
        return SKIP_P && k == 3 ? 4 : k;
    }
    __device__ __forceinline__ void init(const Geo& g, int xa, int ya) {
        const bool lat = g.bcl == JFNK_BC_PERIODIC;
#pragma unroll
        for (int p = 0; p < POS; ++p) {
            const int idx = (int)threadIdx.x + p * NTHR;
            off[p] = 0;
            xyneg[p] = 0u;
            if (idx < MG::P) {
                const int ly = idx / MG::SX, lx = idx - ly * MG::SX;
                int sx, sy;
                const int mx = map3(xa + lx, g.nx, lat, sx), my = map3(ya + ly, g.ny, lat, sy);
                off[p] = my * g.nx + mx;
                unsigned m = 0u;
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    if (odd3(sfield(f), sx, sy, 0, g.bcv)) m |= 1u << f;
                xyneg[p] = m;
            }
        }
    }
    __device__ __forceinline__ void load(const Geo& g, const T* __restrict__ a, const T* __restrict__ b, int z) {
        int sz;
        const int mz = map3(z, g.nz, g.bcv == JFNK_BC_PERIODIC, sz);
        const long long pl = (long long)mz * g.nx * g.ny;
        unsigned m = 0u;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (odd3(sfield(f), 0, 0, sz, g.bcv)) m |= 1u << f;
            const T* base = (f < NS ? a : b) + (long long)sfield(f) * g.npts + pl;
#pragma unroll
            for (int p = 0; p < POS; ++p) r[p][f] = base[off[p]];
        }
        zneg = m;
    }
    __device__ __forceinline__ void store(T* dst) const {
#pragma unroll
        for (int p = 0; p < POS; ++p) {
            const int idx = (int)threadIdx.x + p * NTHR;
            if (idx < MG::P) {
                const unsigned m = xyneg[p] ^ zneg;
#pragma unroll
                for (int f = 0; f < NF; ++f) dst[f * MG::P + idx] = (m >> f) & 1u ? -r[p][f] : r[p][f];
            }
        }
    }
};

// Window accessor: field f at offset (ox, oy, oz) from the thread's point
template <typename T, int TY>
struct Win {
    const T* slot[5];   // planes z-2 .. z+2
    int c;              // in-plane index of the thread's point
    __device__ __forceinline__ T at(int f, int ox, int oy, int oz) const {
        using MG = MarchGeom<TY>;
        return slot[oz + 2][f * MG::P + c + oy * MG::SX + ox];
    }
    __device__ __forceinline__ T d(int f, int a, T ih) const {   // derivative along axis a
        const int ex = a == 0, ey = a == 1, ez = a == 2;
        return d5(at(f, -2 * ex, -2 * ey, -2 * ez), at(f, -ex, -ey, -ez), at(f, ex, ey, ez),
                  at(f, 2 * ex, 2 * ey, 2 * ez), ih);
    }
};

// gradient of the velocity (window fields 0..2) and of theta (window field 3)
template <typename T, int TY>
__device__ __forceinline__ void strain_win(const Geo& g, const Win<T, TY>& w, int f0, T S[6], T th[3]) {
    const T ih[3] = {T(g.idx), T(g.idy), T(g.idz)};
    T gr[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] = w.d(f0 + i, j, ih[j]);
    S[0] = gr[0][0];
    S[1] = gr[1][1];
    S[2] = gr[2][2];
    S[3] = T(0.5) * (gr[0][1] + gr[1][0]);
    S[4] = T(0.5) * (gr[0][2] + gr[2][0]);
    S[5] = T(0.5) * (gr[1][2] + gr[2][1]);
#pragma unroll
    for (int j = 0; j < 3; ++j) th[j] = w.d(f0 + 3, j, ih[j]);
}

// Pass 1: tau (6) and q (3) on the ring-2 extended grid [9][nz+4][ny+4][nx+4],
// or with PAIR their finite-difference differences for (u, v):
// [tau(u + e v) - tau(u)] / e with the stable nu difference.
template <typename T, bool PAIR>
__global__ __launch_bounds__(256) void k3m_derived(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                   double eps_in, const double* __restrict__ eps_dev,
                                                   T* __restrict__ d) {
    constexpr int TY = 8;
    using MG = MarchGeom<TY>;
    constexpr int NF = PAIR ? 8 : 4;
    __shared__ T win[5 * NF * MG::P];
    const int EX = g.nx + 4, EY = g.ny + 4, EZ = g.nz + 4;
    const long long ne = (long long)EX * EY * EZ;
    const int tx = threadIdx.x % kMTX, ty = threadIdx.x / kMTX;
    const int xe = blockIdx.x * kMTX + tx, ye = blockIdx.y * TY + ty;
    const int ze0 = blockIdx.z * kZC, ze1 = min(ze0 + kZC, EZ);
    const bool mine = xe < EX && ye < EY;
    // region origin: grid point (xe0 - 2) - 2 along x, likewise y
    const int xa = blockIdx.x * kMTX - 4, ya = blockIdx.y * TY - 4;
    const T e = PAIR ? T(eps_dev ? *eps_dev : eps_in) : T(0);
    Stager<T, NF, TY, 256, 4, true> st;
    st.init(g, xa, ya);
    // planes z - 2 .. z + 1 of the first point z = ze0 - 2, then z + 2 in flight
    for (int k = 0; k < 4; ++k) {
        st.load(g, u, v, ze0 - 4 + k);
        st.store(win + k * NF * MG::P);
    }
    st.load(g, u, v, ze0);
    for (int ze = ze0; ze < ze1; ++ze) {
        const int z = ze - 2;
        const int r0 = ze - ze0;                 // ring slot of plane z - 2
        st.store(win + ((r0 + 4) % 5) * NF * MG::P);
        __syncthreads();
        if (ze + 1 < ze1) st.load(g, u, v, z + 3);
        if (mine) {
            Win<T, TY> w;
#pragma unroll
            for (int k = 0; k < 5; ++k) w.slot[k] = win + ((r0 + k) % 5) * NF * MG::P;
            w.c = (ty + 2) * MG::SX + tx + 2;
            const long long i = ((long long)ze * EY + ye) * EX + xe;
            if (!PAIR) {
                T S[6], th[3];
                strain_win<T, TY>(g, w, 0, S, th);
                const Coef<T> k = closure3c(g, frob3(S, S));
                const T third = (S[0] + S[1] + S[2]) * T(1.0 / 3.0);
                d[0 * ne + i] = T(2) * k.mh * (S[0] - third);
                d[1 * ne + i] = T(2) * k.mh * (S[1] - third);
                d[2 * ne + i] = T(2) * k.mv * (S[2] - third);
                d[3 * ne + i] = T(2) * k.mh * S[3];
                d[4 * ne + i] = T(2) * k.mv * S[4];
                d[5 * ne + i] = T(2) * k.mv * S[5];
                d[6 * ne + i] = k.hh * th[0];
                d[7 * ne + i] = k.hh * th[1];
                d[8 * ne + i] = k.hv * th[2];
            } else {
                T SU[6], SV[6], tU[3], tV[3];
                strain_win<T, TY>(g, w, 0, SU, tU);
                strain_win<T, TY>(g, w, 4, SV, tV);
                const Coef<T> ka = closure3c(g, frob3(SU, SU));
                T SW[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) SW[k] = SU[k] + e * SV[k];
                Coef<T> dk = {T(0), T(0), T(0), T(0)};
                if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
                    const T den = sqrt(frob3(SU, SU)) + sqrt(frob3(SW, SW));
                    const T num = T(2) * frob3(SU, SV) + e * frob3(SV, SV);
                    if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
                        const T dnu = den > T(0) ? T(g.smag) * T(1.4142135623730951) * num / den : T(0);
                        const T dkth = dnu * T(g.inv_pr);
                        dk = {dnu, dnu, dkth, dkth};
                    } else {
                        dk = deardorff_diff(g, T(sqrt(frob3(SU, SU))), den > T(0) ? num / den : T(0), e);
                    }
                }
                const T trw = (SW[0] + SW[1] + SW[2]) * T(1.0 / 3.0), trv = (SV[0] + SV[1] + SV[2]) * T(1.0 / 3.0);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const T dw = k < 3 ? SW[k] - trw : SW[k];
                    const T dv = k < 3 ? SV[k] - trv : SV[k];
                    d[k * ne + i] = T(2) * (vert3(k) ? dk.mv : dk.mh) * dw + T(2) * (vert3(k) ? ka.mv : ka.mh) * dv;
                }
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    d[(6 + j) * ne + i] = (j == 2 ? dk.hv : dk.hh) * (tU[j] + e * tV[j]) + (j == 2 ? ka.hv : ka.hh) * tV[j];
            }
        }
        __syncthreads();
    }
}

// In-plane derived components staged per plane: xx, yy, xy, xz, yz, qx, qy
// (slots 0..6); the z-derivatives take xz, yz, zz, qz from a per-thread queue.
__device__ __forceinline__ int dplane_slot(int comp) {
    return comp == 0 ? 0 : comp == 1 ? 1 : comp == 3 ? 2 : comp == 4 ? 3 : comp == 5 ? 4 : comp == 6 ? 5 : 6;
}
// five consecutive planes of one value, oldest first
template <typename T> struct Q5 {
    T m2, m1, c0, p1, p2;
    __device__ __forceinline__ void push(T x) {
        m2 = m1;
        m1 = c0;
        c0 = p1;
        p1 = p2;
        p2 = x;
    }
};
constexpr int kDPlane[7] = {0, 1, 3, 4, 5, 6, 7};
constexpr int kDQueue[4] = {4, 5, 2, 8};

// Pass 2 (per grid point).  MODE 0: out = F (what 0), 2u/dt + F (1) or
// 2u/dt - F - f (2) of state u; MODE 1: Jv = 2v/dt - [F(u + e v) - F(u)]/e with
// the bilinear terms expanded (d holds the derived differences).
template <typename T, int MODE, int TY>
__global__ __launch_bounds__(256) void k3m_point(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                 double eps_in, const double* __restrict__ eps_dev,
                                                 const T* __restrict__ d, const T* __restrict__ f,
                                                 T* __restrict__ out, int what) {
    using MG = MarchGeom<TY>;
    constexpr int NF = MODE == 1 ? 10 : 5;
    __shared__ T win[5 * NF * MG::P];
    __shared__ T dpl[7 * MG::P];
    const int EX = g.nx + 4, EY = g.ny + 4;
    const long long ne = (long long)EX * EY * (g.nz + 4);
    const long long np = g.npts;
    constexpr int NTHR = kMTX * TY;
    const int tx = threadIdx.x % kMTX, ty = threadIdx.x / kMTX;
    const int x = blockIdx.x * kMTX + tx, y = blockIdx.y * TY + ty;
    const int z0 = blockIdx.z * kZC, z1 = min(z0 + kZC, g.nz);
    const bool mine = x < g.nx && y < g.ny;
    const int xa = blockIdx.x * kMTX - 2, ya = blockIdx.y * TY - 2;
    const T e = MODE == 1 ? T(eps_dev ? *eps_dev : eps_in) : T(0);
    const T ih[3] = {T(g.idx), T(g.idy), T(g.idz)};
    // clamped ext-grid columns (points outside the grid never read them)
    auto dcol = [&](int xx, int yy) {
        return (long long)min(max(yy + 2, 0), EY - 1) * EX + min(max(xx + 2, 0), EX - 1);
    };
    const long long pe = (long long)EX * EY;
    const long long mycol = dcol(x, y);
    // in-plane derived components of one plane over the region, one plane ahead
    // (fixed positions per thread as in Stager)
    constexpr int DPOS = (MG::P + NTHR - 1) / NTHR;
    int doff[DPOS];
#pragma unroll
    for (int p = 0; p < DPOS; ++p) {
        const int idx = min((int)threadIdx.x + p * NTHR, MG::P - 1);
        const int ly = idx / MG::SX, lx = idx - ly * MG::SX;
        doff[p] = (int)dcol(xa + lx, ya + ly);
    }
    T dr[DPOS][7];
    auto dload = [&](int zz) {
#pragma unroll
        for (int sl = 0; sl < 7; ++sl) {
            const T* base = d + kDPlane[sl] * ne + (zz + 2) * pe;
#pragma unroll
            for (int p = 0; p < DPOS; ++p) dr[p][sl] = base[doff[p]];
        }
    };
    // z queue of xz, yz, zz, qz at z - 2 .. z + 2 (named registers), the next
    // plane in qn
    Q5<T> q[4];
    T qn[4];
    auto qload = [&](int zz) {
#pragma unroll
        for (int c = 0; c < 4; ++c) qn[c] = d[kDQueue[c] * ne + (zz + 2) * pe + mycol];
    };
    Stager<T, NF, TY, NTHR, 5, false> st;
    st.init(g, xa, ya);
    for (int k = 0; k < 4; ++k) {
        st.load(g, u, v, z0 - 2 + k);
        st.store(win + k * NF * MG::P);
        qload(z0 - 2 + k);
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c].push(qn[c]);
    }
    st.load(g, u, v, z0 + 2);
    dload(z0);
    qload(z0 + 2);
    for (int z = z0; z < z1; ++z) {
        const int r0 = z - z0;
        st.store(win + ((r0 + 4) % 5) * NF * MG::P);
#pragma unroll
        for (int p = 0; p < DPOS; ++p) {
            const int idx = (int)threadIdx.x + p * NTHR;
            if (idx < MG::P) {
#pragma unroll
                for (int sl = 0; sl < 7; ++sl) dpl[sl * MG::P + idx] = dr[p][sl];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c].push(qn[c]);
        __syncthreads();
        if (z + 1 < z1) {
            st.load(g, u, v, z + 3);
            dload(z + 1);
            qload(z + 3);
        }
        if (mine) {
            Win<T, TY> wa, wb;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                wa.slot[k] = win + ((r0 + k) % 5) * NF * MG::P;
                wb.slot[k] = wa.slot[k] + 5 * MG::P;
            }
            wa.c = wb.c = (ty + 2) * MG::SX + tx + 2;
            // derivative of derived component comp along axis j at the point
            auto dd = [&](int comp, int j) -> T {
                if (j == 2) {
                    const Q5<T>& qq = comp == 4 ? q[0] : comp == 5 ? q[1] : comp == 2 ? q[2] : q[3];
                    return d5(qq.m2, qq.m1, qq.p1, qq.p2, ih[2]);
                }
                const T* pl = dpl + dplane_slot(comp) * MG::P + wa.c;
                const int st = j == 0 ? 1 : MG::SX;
                return d5(pl[-2 * st], pl[-st], pl[st], pl[2 * st], ih[j]);
            };
            const long long i = ((long long)z * g.ny + y) * g.nx + x;
            const T th0 = T(g.theta0);
            const T* pb = Bg<T>::pbar(g);
            const T* dpb = Bg<T>::dpbar(g);
            if (MODE == 0) {
                T val[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) val[k] = wa.at(k, 0, 0, 0);
                T Fv[5] = {0, 0, 0, 0, 0};
                if (g.convection) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int ex = j == 0, ey = j == 1, ez = j == 2;
                        const T am2 = wa.at(j, -2 * ex, -2 * ey, -2 * ez), am1 = wa.at(j, -ex, -ey, -ez);
                        const T ap1 = wa.at(j, ex, ey, ez), ap2 = wa.at(j, 2 * ex, 2 * ey, 2 * ez);
#pragma unroll
                        for (int k = 0; k < 5; ++k) {
                            const T pm2 = wa.at(k, -2 * ex, -2 * ey, -2 * ez), pm1 = wa.at(k, -ex, -ey, -ez);
                            const T pp1 = wa.at(k, ex, ey, ez), pp2 = wa.at(k, 2 * ex, 2 * ey, 2 * ez);
                            const T flux = d5(am2 * pm2, am1 * pm1, ap1 * pp1, ap2 * pp2, ih[j]);
                            const T adv = val[j] * d5(pm2, pm1, pp1, pp2, ih[j]);
                            Fv[k] -= T(0.5) * (flux + adv);
                        }
                    }
                }
                T div = T(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Fv[c] -= th0 * wa.d(3, c, ih[c]);
                    div += wa.d(c, c, ih[c]);
#pragma unroll
                    for (int j = 0; j < 3; ++j) Fv[c] += dd(tix(c, j), j);
                }
                Fv[2] += T(g.g_theta0) * val[4];
                if (g.energy_test)
                    Fv[3] -= T(g.kappa_cp) * div;
                else
                    Fv[3] -= val[2] * dpb[z] + T(g.kappa) * (pb[z] + val[3]) * div;
#pragma unroll
                for (int j = 0; j < 3; ++j) Fv[4] += dd(6 + j, j);
                Fv[4] -= T(g.beta) * val[2];
                if (z == 0 && !g.energy_test) Fv[4] += Bg<T>::sflux(g)[(long long)y * g.nx + x];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    T r;
                    if (what == 0) r = Fv[k];
                    else if (what == 1) r = T(g.two_dt) * val[k] + Fv[k];
                    else r = T(g.two_dt) * val[k] - Fv[k] - (f ? f[k * np + i] : T(0));
                    out[k * np + i] = r;
                }
            } else {
                T A[5], B[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    A[k] = wa.at(k, 0, 0, 0);
                    B[k] = wb.at(k, 0, 0, 0);
                }
                T dF[5] = {0, 0, 0, 0, 0};
                if (g.convection) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int ex = j == 0, ey = j == 1, ez = j == 2;
                        const int ox[4] = {-2, -1, 1, 2};
                        T au[4], bv[4];
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq) {
                            au[qq] = wa.at(j, ox[qq] * ex, ox[qq] * ey, ox[qq] * ez);
                            bv[qq] = wb.at(j, ox[qq] * ex, ox[qq] * ey, ox[qq] * ez);
                        }
#pragma unroll
                        for (int k = 0; k < 5; ++k) {
                            T pa[4], pbv[4], pr[4];
#pragma unroll
                            for (int qq = 0; qq < 4; ++qq) {
                                pa[qq] = wa.at(k, ox[qq] * ex, ox[qq] * ey, ox[qq] * ez);
                                pbv[qq] = wb.at(k, ox[qq] * ex, ox[qq] * ey, ox[qq] * ez);
                                pr[qq] = au[qq] * pbv[qq] + bv[qq] * (pa[qq] + e * pbv[qq]);
                            }
                            const T flux = d5(pr[0], pr[1], pr[2], pr[3], ih[j]);
                            const T dA = d5(pa[0], pa[1], pa[2], pa[3], ih[j]);
                            const T dB = d5(pbv[0], pbv[1], pbv[2], pbv[3], ih[j]);
                            const T adv = A[j] * dB + B[j] * (dA + e * dB);
                            dF[k] -= T(0.5) * (flux + adv);
                        }
                    }
                }
                T divA = T(0), divB = T(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dF[c] -= th0 * wb.d(3, c, ih[c]);
                    divA += wa.d(c, c, ih[c]);
                    divB += wb.d(c, c, ih[c]);
#pragma unroll
                    for (int j = 0; j < 3; ++j) dF[c] += dd(tix(c, j), j);
                }
                dF[2] += T(g.g_theta0) * B[4];
                if (g.energy_test)
                    dF[3] -= T(g.kappa_cp) * divB;
                else
                    dF[3] -= B[2] * dpb[z] + T(g.kappa) * ((pb[z] + A[3]) * divB + B[3] * divA + e * B[3] * divB);
#pragma unroll
                for (int j = 0; j < 3; ++j) dF[4] += dd(6 + j, j);
                dF[4] -= T(g.beta) * B[2];
                const T tdt = T(g.two_dt);
#pragma unroll
                for (int k = 0; k < 5; ++k) out[k * np + i] = tdt * B[k] - dF[k];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Single-launch 3D Jv (the stable finite-difference quotient of Eq. 9, FP32).
// A workgroup owns 32 x TY columns and marches along z; at step s it forms the
// differences of the stress and heat flux (the derived quantities) at plane
// s + 2 over the columns grown by 2, and Jv at plane s:
//  - 32 x TY own-column threads hold their column's planes s-2 .. s+4 of A = u
//    and B = v (p: s-2 .. s+2) in registers; 256 ring threads (waves of their
//    own, so a SIMD runs two own-column waves and one ring wave) hold a
//    column of the ring of 2 around the tile (planes s .. s+4, p at s) and
//    one of the ring between 2 and 4 (plane s+2), load them, stage them in
//    LDS and form the ring's derived quantities;
//  - in-plane neighbours come from LDS: plane s+2 over the columns grown by 4
//    (gradients of the derived stage) and plane s over the columns grown by 2
//    as W = A + e B and B (convection, pressure gradient, divergence);
//  - the in-plane derived components (xx, yy, xy, xz, yz, qx, qy) of planes
//    s .. s+2 live in an LDS ring of three planes, the own columns' vertical
//    ones (xz, yz, zz, qz) of planes s-2 .. s+2 in an LDS ring of five planes
//    that only the column's thread touches.
// Every state value comes from HBM once per workgroup (plus the halos) and Jv
// is the only array written: 3 n_f values per point against the two-pass
// form's 9 extra components written and read back.
// ---------------------------------------------------------------------------
template <int TY> struct FusedGeom {
    static constexpr int TX = 32, NT = TX * TY;
    static constexpr int SX2 = TX + 4, SY2 = TY + 4, P2 = SX2 * SY2;   // the columns grown by 2
    static constexpr int SX4 = TX + 8, SY4 = TY + 8, P4 = SX4 * SY4;   // grown by 4
    static constexpr int NRIM2 = P2 - NT, NRIM4 = P4 - P2;
};

// r-th column of the ring of 2 around the tile, in the coordinates of the
// columns grown by 2: two full rows below, two above, then two columns each side
template <int TY>
__device__ __forceinline__ void fused_rim2(int r, int& lx, int& ly) {
    using FG = FusedGeom<TY>;
    constexpr int row2 = 2 * FG::SX2;
    if (r < row2) {
        ly = r / FG::SX2;
        lx = r - ly * FG::SX2;
    } else if (r < 2 * row2) {
        r -= row2;
        ly = TY + 2 + r / FG::SX2;
        lx = r - (ly - TY - 2) * FG::SX2;
    } else {
        r -= 2 * row2;
        ly = 2 + (r >> 2);
        const int c = r & 3;
        lx = c < 2 ? c : FG::TX + c;
    }
}

// r-th column of the ring between the columns grown by 2 and by 4, in the
// coordinates of the columns grown by 4
template <int TY>
__device__ __forceinline__ void fused_rim4(int r, int& lx, int& ly) {
    using FG = FusedGeom<TY>;
    constexpr int row2 = 2 * FG::SX4;
    if (r < row2) {
        ly = r / FG::SX4;
        lx = r - ly * FG::SX4;
    } else if (r < 2 * row2) {
        r -= row2;
        ly = FG::SY4 - 2 + r / FG::SX4;
        lx = r - (ly - FG::SY4 + 2) * FG::SX4;
    } else {
        r -= 2 * row2;
        ly = 2 + (r >> 2);
        const int c = r & 3;
        lx = c < 2 ? c : FG::SX4 - 4 + c;
    }
}

// fields of the derived stage: (u, v, w, theta) of A, then of B; state indices
__device__ __forceinline__ constexpr int fused_sf(int k) { return k == 3 ? 4 : k; }

// Derived quantities of the pair (A, B) at one column of plane za: the stable
// differences [tau(A + e B) - tau(A)] / e and [q(A + e B) - q(A)] / e (as in
// k3m_derived).  L points at the column in the LDS plane za over the columns
// grown by 4 (fields A u, v, w, theta, B u, v, w, theta); q(k, f) is field f of
// the column at plane za - 2 + k.  out: xx, yy, zz, xy, xz, yz, qx, qy, qz.
template <int TY, typename ZQ>
__device__ __forceinline__ void fused_derived(const Geo& g, const float* __restrict__ L, ZQ q, float e,
                                              float ihx, float ihy, float ihz, float out[9]) {
    using FG = FusedGeom<TY>;
    constexpr int P = FG::P4, S = FG::SX4;
    float gA[3][3], gB[3][3], tA[3], tB[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = i + 4 * h;
            const float* c = L + f * P;
            const float dx = d5(c[-2], c[-1], c[1], c[2], ihx);
            const float dy = d5(c[-2 * S], c[-S], c[S], c[2 * S], ihy);
            const float dz = d5(q(0, f), q(1, f), q(3, f), q(4, f), ihz);
            float* gr = i < 3 ? (h ? gB[i] : gA[i]) : (h ? tB : tA);
            gr[0] = dx;
            gr[1] = dy;
            gr[2] = dz;
        }
    }
    float SA[6], SB[6], SW[6];
    SA[0] = gA[0][0], SA[1] = gA[1][1], SA[2] = gA[2][2];
    SA[3] = 0.5f * (gA[0][1] + gA[1][0]), SA[4] = 0.5f * (gA[0][2] + gA[2][0]), SA[5] = 0.5f * (gA[1][2] + gA[2][1]);
    SB[0] = gB[0][0], SB[1] = gB[1][1], SB[2] = gB[2][2];
    SB[3] = 0.5f * (gB[0][1] + gB[1][0]), SB[4] = 0.5f * (gB[0][2] + gB[2][0]), SB[5] = 0.5f * (gB[1][2] + gB[2][1]);
#pragma unroll
    for (int k = 0; k < 6; ++k) SW[k] = SA[k] + e * SB[k];
    Coef<float> ka = {0.f, 0.f, 0.f, 0.f}, dk = {0.f, 0.f, 0.f, 0.f};
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
        // hardware square root and reciprocal (1 ulp): well inside the FP32 parity bar
        const float ma = __builtin_amdgcn_sqrtf(frob3(SA, SA)), mw = __builtin_amdgcn_sqrtf(frob3(SW, SW));
        const float den = ma + mw;
        const float num = 2.f * frob3(SA, SB) + e * frob3(SB, SB);
        if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
            const float c = g.f.smag_s2;
            const float nu = c * ma, dnu = den > 0.f ? c * num * __builtin_amdgcn_rcpf(den) : 0.f;
            const float ip = g.f.inv_pr;
            ka = {nu, nu, nu * ip, nu * ip};
            dk = {dnu, dnu, dnu * ip, dnu * ip};
        } else {
            ka = deardorff_coef(g, ma);
            dk = deardorff_diff(g, ma, den > 0.f ? num / den : 0.f, e);
        }
    } else if (g.closure == JFNK_CLOSURE_CONST_K) {
        ka = {float(g.k_m), float(g.k_m), float(g.k_h), float(g.k_h)};
    }
    const float trw = (SW[0] + SW[1] + SW[2]) * (1.f / 3.f), trb = (SB[0] + SB[1] + SB[2]) * (1.f / 3.f);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float dw = k < 3 ? SW[k] - trw : SW[k];
        const float db = k < 3 ? SB[k] - trb : SB[k];
        out[k] = 2.f * ((vert3(k) ? dk.mv : dk.mh) * dw + (vert3(k) ? ka.mv : ka.mh) * db);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        out[6 + j] = (j == 2 ? dk.hv : dk.hh) * (tA[j] + e * tB[j]) + (j == 2 ? ka.hv : ka.hh) * tB[j];
}

// The kernel: 32 x TY + 256 threads, roles by wave (own columns first).
template <int TY>
__global__ __launch_bounds__(32 * TY + 256) void k3f_jv(Geo g, const float* __restrict__ u,
                                                         const float* __restrict__ v, double eps_in,
                                                         const double* __restrict__ eps_dev,
                                                         float* __restrict__ out, int kzc) {
    using FG = FusedGeom<TY>;
    static_assert(FG::NRIM2 <= 256 && FG::NRIM4 <= 256, "the ring columns exceed the ring threads");
    __shared__ float L4[8 * FG::P4];        // plane s+2 over the columns grown by 4
    __shared__ float L2[10 * FG::P2];       // plane s over the columns grown by 2: W = A + e B, then B (state order)
    __shared__ float RG[3 * 7 * FG::P2];    // in-plane derived components of planes s .. s+2
    __shared__ float TQ[5 * 4 * FG::NT];    // own columns: xz, yz, zz, qz of planes s-2 .. s+2 (slot = plane mod 5)
    const int tid = threadIdx.x;
    const bool own = tid < FG::NT;          // uniform per wave
    const int rt = tid - FG::NT;            // ring thread index
    const int tx = tid & 31, ty = tid >> 5;
    const int gx = (g.nx + 31) / 32, gy = (g.ny + TY - 1) / TY;
    const int nblk = (int)gridDim.x;
    int t = (int)blockIdx.x;
    if (nblk % 8 == 0) t = (t % 8) * (nblk / 8) + t / 8;
    const int bx = t % gx, by = (t / gx) % gy, bz = t / (gx * gy);
    const int x0 = bx * 32, y0 = by * TY;
    const int z0 = bz * kzc, z1 = min(z0 + kzc, g.nz);
    const bool lat = g.bcl == JFNK_BC_PERIODIC, vper = g.bcv == JFNK_BC_PERIODIC;
    const long long np = g.npts, nxy = (long long)g.nx * g.ny;
    const float e = (float)(eps_dev ? *eps_dev : eps_in);
    const float ihx = g.f.idx, ihy = g.f.idy, ihz = g.f.idz;

    auto setup = [&](int gx, int gy, int& off, unsigned& neg) {
        int sx, sy;
        const int mx = map3(gx, g.nx, lat, sx), my = map3(gy, g.ny, lat, sy);
        off = my * g.nx + mx;
        unsigned m = 0u;
#pragma unroll
        for (int f = 0; f < 5; ++f)
            if (odd3(f, sx, sy, 0, g.bcv)) m |= 1u << f;
        neg = m;
    };
    auto zmap = [&](int z, long long& pl, unsigned& neg) {
        if (z >= 0 && z < g.nz) {   // interior plane: no reflection
            pl = (long long)z * nxy;
            neg = 0u;
            return;
        }
        int sz;
        const int mz = map3(z, g.nz, vper, sz);
        pl = (long long)mz * nxy;
        unsigned m = 0u;
#pragma unroll
        for (int f = 0; f < 5; ++f)
            if (odd3(f, 0, 0, sz, g.bcv)) m |= 1u << f;
        neg = m;
    };
    auto sgn = [](float x, unsigned neg, int f) { return (neg >> f) & 1u ? -x : x; };
    auto ld8 = [&](int off, long long pl, float (&r)[8]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r[k] = u[fused_sf(k) * np + pl + off];
            r[4 + k] = v[fused_sf(k) * np + pl + off];
        }
    };
    auto ldp = [&](int off, long long pl, float (&r)[2]) {
        r[0] = u[3 * np + pl + off];
        r[1] = v[3 * np + pl + off];
    };
    auto fix8 = [&](float (&r)[8], unsigned neg) {
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = sgn(r[k], neg, fused_sf(k & 3));
    };
    auto fixp = [&](float (&r)[2], unsigned neg) {
        r[0] = sgn(r[0], neg, 3);
        r[1] = sgn(r[1], neg, 3);
    };

    // own thread: its column; ring thread: a ring-of-2 column (has1) and a
    // ring-of-4 column (has4)
    const int px = x0 + tx, py = y0 + ty;
    const bool mine = own && px < g.nx && py < g.ny;
    const bool has1 = !own && rt < FG::NRIM2, has4 = !own && rt < FG::NRIM4;
    int lx1 = 0, ly1 = 0, lx4 = 0, ly4 = 0;
    if (has1) fused_rim2<TY>(rt, lx1, ly1);
    if (has4) fused_rim4<TY>(rt, lx4, ly4);
    int offA, offB = 0;   // own: the column; ring: the ring-of-2 column (A) and the ring-of-4 column (B)
    unsigned negA, negB = 0u;
    if (own)
        setup(px, py, offA, negA);
    else {
        setup(x0 - 2 + lx1, y0 - 2 + ly1, offA, negA);
        setup(x0 - 4 + lx4, y0 - 4 + ly4, offB, negB);
    }
    const int c2 = own ? (ty + 2) * FG::SX2 + tx + 2 : ly1 * FG::SX2 + lx1;
    const int c4 = own ? (ty + 4) * FG::SX4 + tx + 4 : (ly1 + 2) * FG::SX4 + lx1 + 2;
    const int c4x = ly4 * FG::SX4 + lx4;

    // register queues, one layout for both roles so that both advance them
    // the same way (slot 0 oldest): Q[2..6] the column's planes s .. s+4 and
    // P[2] its p at plane s; own columns also Q[0], Q[1] (planes s-2, s-1)
    // and P[0], P[1], P[3], P[4] (p at s-2 .. s+2); ring threads keep their
    // ring-of-4 column's plane s+2 in Q[0] and receive its next plane in Q[1]
    // and the next p of their ring-of-2 column in P[3] (each moved down one
    // slot by the advance)
    float Q[7][8];
    float P[5][2];
    const int sb = z0 - 4;   // first step: the derived stage starts at plane z0 - 2
    {
        long long pl;
        unsigned nz_;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            zmap(sb - 2 + k, pl, nz_);
            if (own || k >= 2) {
                ld8(offA, pl, Q[k]);
                fix8(Q[k], negA ^ nz_);
            }
            if (own ? k < 5 : k == 2) {
                ldp(offA, pl, P[k]);
                fixp(P[k], negA ^ nz_);
            }
            if (!own && k == 4) {
                ld8(offB, pl, Q[0]);   // ring-of-4 column, plane sb + 2
                fix8(Q[0], negB ^ nz_);
            }
        }
    }
    const float* pb = g.pbar32;
    const float* dpb = g.dpbar32;
    const float th0 = g.f.theta0, kap = g.f.kappa, kcp = g.f.kappa_cp;
    const float gth = g.f.g_theta0, bet = g.f.beta, tdt = g.f.two_dt;
    int r5 = (sb + 10) % 5, r3 = (sb + 6) % 3;   // slots of plane s
    auto m5 = [](int a) { return a >= 5 ? a - 5 : a; };
    auto m3 = [](int a) { return a >= 3 ? a - 3 : a; };
    float* tq = TQ + tid;   // own column's slot base (stride NT per component, 4 NT per plane)

    for (int s = sb; s < z1; ++s) {
        // (1) LDS: plane s+2 over the columns grown by 4, plane s over those grown by 2
        {
            // plane s+2 of the column to L4, plane s (W = A + e B and B) to L2
            auto put = [&](const float (&q2)[8], const float (&q0)[8], const float (&p0)[2]) {
#pragma unroll
                for (int k = 0; k < 8; ++k) L4[k * FG::P4 + c4] = q2[k];
                const float a[10] = {q0[0] + e * q0[4], q0[1] + e * q0[5], q0[2] + e * q0[6], p0[0] + e * p0[1],
                                     q0[3] + e * q0[7], q0[4], q0[5], q0[6], p0[1], q0[7]};
#pragma unroll
                for (int k = 0; k < 10; ++k) L2[k * FG::P2 + c2] = a[k];
            };
            if (own || has1) put(Q[4], Q[2], P[2]);
            if (has4) {
#pragma unroll
                for (int k = 0; k < 8; ++k) L4[k * FG::P4 + c4x] = Q[0][k];
            }
        }
        __syncthreads();
        // (2) loads for the next step (consumed after the closing barrier)
        const bool more = s + 1 < z1;
        float n0[8], np0[2];
        unsigned m0 = 0u, mp0 = 0u, m1 = 0u, m4 = 0u;
        if (more) {
            long long pl;
            unsigned zn;
            zmap(s + 5, pl, zn);   // the column's plane s+5
            if (own || has1) ld8(offA, pl, n0);
            m0 = negA ^ zn;
            if (own) {
                zmap(s + 3, pl, zn);
                ldp(offA, pl, np0);
                mp0 = negA ^ zn;
            } else {
                zmap(s + 1, pl, zn);
                if (has1) ldp(offA, pl, P[3]);   // ring-of-2 p at plane s+1
                m1 = negA ^ zn;
                zmap(s + 3, pl, zn);
                if (has4) ld8(offB, pl, Q[1]);   // ring-of-4 plane s+3
                m4 = negB ^ zn;
            }
        }
        // (3) derived stage at plane s+2 (own and ring-of-2 columns)
        const int slotA = m3(r3 + 2);
        if (own || has1) {
            float d[9];
            fused_derived<TY>(g, L4 + c4, [&](int k, int f) { return Q[2 + k][f]; }, e, ihx, ihy, ihz, d);
            float* rg = RG + slotA * 7 * FG::P2 + c2;
            rg[0 * FG::P2] = d[0];
            rg[1 * FG::P2] = d[1];
            rg[2 * FG::P2] = d[3];
            rg[3 * FG::P2] = d[4];
            rg[4 * FG::P2] = d[5];
            rg[5 * FG::P2] = d[6];
            rg[6 * FG::P2] = d[7];
            if (own) {
                float* w = tq + m5(r5 + 2) * 4 * FG::NT;   // plane s+2
                w[0 * FG::NT] = d[4];
                w[1 * FG::NT] = d[5];
                w[2 * FG::NT] = d[2];
                w[3 * FG::NT] = d[8];
            }
        }
        // (4) Jv at plane s (its derived ring plane was written two steps ago)
        if (s >= z0 && mine) {
            const float* l2 = L2 + c2;
            const float Ac[5] = {Q[2][0], Q[2][1], Q[2][2], P[2][0], Q[2][3]};
            const float Bc[5] = {Q[2][4], Q[2][5], Q[2][6], P[2][1], Q[2][7]};
            const float ih[2] = {ihx, ihy};
            float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            float divB = 0.f, divW = 0.f, gp[3];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int st = j == 0 ? 1 : FG::SX2;
                auto tw = [&](int f, int k) { return l2[f * FG::P2 + (k < 2 ? k - 2 : k - 1) * st]; };
                auto tb = [&](int f, int k) { return l2[(5 + f) * FG::P2 + (k < 2 ? k - 2 : k - 1) * st]; };
                float aj[4], bj[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    bj[k] = tb(j, k);
                    aj[k] = tw(j, k) - e * bj[k];
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    float w[4], b[4], pr[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        w[k] = tw(f, k);
                        b[k] = f == j ? bj[k] : tb(f, k);
                        pr[k] = aj[k] * b[k] + bj[k] * w[k];
                    }
                    const float dB = d5(b[0], b[1], b[2], b[3], ih[j]);
                    const float dW = d5(w[0], w[1], w[2], w[3], ih[j]);
                    if (f == j) {
                        divB += dB;
                        divW += dW;
                    }
                    if (f == 3) gp[j] = dB;
                    if (g.convection) acc[f] += d5(pr[0], pr[1], pr[2], pr[3], ih[j]) + Ac[j] * dB + Bc[j] * dW;
                }
            }
            {
                constexpr int oz[4] = {0, 1, 3, 4};
                auto za = [&](int f, int k) { return f == 3 ? P[oz[k]][0] : Q[oz[k]][f == 4 ? 3 : f]; };
                auto zb = [&](int f, int k) { return f == 3 ? P[oz[k]][1] : Q[oz[k]][(f == 4 ? 3 : f) + 4]; };
                float wz[4], bz[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    bz[k] = zb(2, k);
                    wz[k] = za(2, k) + e * bz[k];
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    float a[4], b[4], pr[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        a[k] = za(f, k);
                        b[k] = zb(f, k);
                        pr[k] = wz[k] * b[k] + bz[k] * a[k];
                    }
                    const float dB = d5(b[0], b[1], b[2], b[3], ihz);
                    const float dW = d5(a[0], a[1], a[2], a[3], ihz) + e * dB;
                    if (f == 2) {
                        divB += dB;
                        divW += dW;
                    }
                    if (f == 3) gp[2] = dB;
                    if (g.convection) acc[f] += d5(pr[0], pr[1], pr[2], pr[3], ihz) + Ac[2] * dB + Bc[2] * dW;
                }
            }
            // divergences of the stress and heat-flux differences
            const float* rg = RG + r3 * 7 * FG::P2 + c2;
            auto Dx = [&](int c) {
                const float* r = rg + c * FG::P2;
                return d5(r[-2], r[-1], r[1], r[2], ihx);
            };
            auto Dy = [&](int c) {
                const float* r = rg + c * FG::P2;
                return d5(r[-2 * FG::SX2], r[-FG::SX2], r[FG::SX2], r[2 * FG::SX2], ihy);
            };
            const int sl0 = r5 * 4 * FG::NT, slm2 = m5(r5 + 3) * 4 * FG::NT, slm1 = m5(r5 + 4) * 4 * FG::NT,
                      slp1 = m5(r5 + 1) * 4 * FG::NT, slp2 = m5(r5 + 2) * 4 * FG::NT;
            (void)sl0;
            auto Dz = [&](int c) {
                return d5(tq[slm2 + c * FG::NT], tq[slm1 + c * FG::NT], tq[slp1 + c * FG::NT],
                          tq[slp2 + c * FG::NT], ihz);
            };
            float dF[5];
            dF[0] = -0.5f * acc[0] - th0 * gp[0] + Dx(0) + Dy(2) + Dz(0);
            dF[1] = -0.5f * acc[1] - th0 * gp[1] + Dx(2) + Dy(1) + Dz(1);
            dF[2] = -0.5f * acc[2] - th0 * gp[2] + Dx(3) + Dy(4) + Dz(2) + gth * Bc[4];
            if (g.energy_test)
                dF[3] = -0.5f * acc[3] - kcp * divB;
            else
                dF[3] = -0.5f * acc[3] - (Bc[2] * dpb[s] + kap * ((pb[s] + Ac[3]) * divB + Bc[3] * divW));
            dF[4] = -0.5f * acc[4] + Dx(5) + Dy(6) + Dz(3) - bet * Bc[2];
            const long long i = (long long)s * nxy + (long long)py * g.nx + px;
#pragma unroll
            for (int k = 0; k < 5; ++k) out[k * np + i] = tdt * Bc[k] - dF[k];
        }
        __syncthreads();
        // (5) advance the queues by one plane
        if (more) {
            fix8(n0, m0);
            fixp(np0, mp0);
            if (!own) {
                fix8(Q[1], m4);
                fixp(P[3], m1);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k)
#pragma unroll
                for (int c = 0; c < 8; ++c) Q[k][c] = Q[k + 1][c];
#pragma unroll
            for (int c = 0; c < 8; ++c) Q[6][c] = n0[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                P[k][0] = P[k + 1][0];
                P[k][1] = P[k + 1][1];
            }
            P[4][0] = np0[0];
            P[4][1] = np0[1];
        }
        r5 = r5 == 4 ? 0 : r5 + 1;
        r3 = r3 == 2 ? 0 : r3 + 1;
    }
}

// frozen coefficients of the preconditioner from the frozen viscosity (for the
// anisotropic closure the Smagorinsky nu, |S| = nu dd_inv_nu)
template <typename T>
__device__ __forceinline__ Coef<T> pc_k3(const Geo& g, T nu_pt) {
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
        const T kth = nu_pt * T(g.inv_pr);
        return {nu_pt, nu_pt, kth, kth};
    }
    if (g.closure == JFNK_CLOSURE_CONST_K) return {T(g.k_m), T(g.k_m), T(g.k_h), T(g.k_h)};
    if (g.closure == JFNK_CLOSURE_DEARDORFF) return deardorff_coef(g, nu_pt * T(g.dd_inv_nu));
    return {T(0), T(0), T(0), T(0)};
}

// diagonal of a field block: 2/dt + 2 sum c^2 (K_h (1/dx^2 + 1/dy^2) + K_v/dz^2); one K
// times sum 1/h^2 for the isotropic closures
template <typename T>
__device__ __forceinline__ T pc_diag3(const Geo& g, T kh, T kv) {
    const T cD = T(65.0 / 72.0);
    if (g.closure == JFNK_CLOSURE_DEARDORFF)
        return T(g.two_dt) + cD * (kh * T(g.idx * g.idx + g.idy * g.idy) + kv * T(g.idz * g.idz));
    return T(g.two_dt) + cD * kh * T(g.idx * g.idx + g.idy * g.idy + g.idz * g.idz);
}

template <typename T>
__device__ __forceinline__ T nuext(const Geo& g, const T* __restrict__ nu, int x, int y, int z) {
    const long long ex = g.nx + 4, ey = g.ny + 4;
    return nu[((long long)(z + 2) * ey + (y + 2)) * ex + (x + 2)];
}

// Shift a register queue one place towards the front and append v.
template <typename T, int N>
__device__ __forceinline__ void qpush(T (&q)[N], T v) {
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) q[i] = q[i + 1];
    q[N - 1] = v;
}

// ---------------------------------------------------------------------------
// z-marching Jacobi sweep of the 3D field-block preconditioner.  A workgroup
// owns 32 x 8 columns and walks a chunk of kZC planes.  In-plane neighbours
// come from LDS: the iterate with a halo of 4 (for K D z at +-2), the horizontal
// velocity and the frozen viscosity with a halo of 2; the fluxes K D_x z and
// K D_y z of the plane are formed once in LDS.  Along z every thread keeps its
// own column in registers: the iterate over 7 planes (z-2 .. z+4), w over 5 and
// the fluxes K D_z z over 5.  Same arithmetic as the per-point sweep it replaces.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k3m_pc_sweep(Geo g, const T* __restrict__ u, const T* __restrict__ nu,
                                                    const T* __restrict__ r, const T* __restrict__ zin,
                                                    T* __restrict__ zout, EpsArgs ea) {
    constexpr int TY = 8, NTHR = kMTX * TY;
    using ZG = MarchGeom<TY, 4>;              // iterate plane, halo 4
    using AG = MarchGeom<TY, 2>;              // velocity and viscosity plane, halo 2
    constexpr int FXN = AG::SX * TY, FYN = kMTX * AG::SY;
    __shared__ T sz[5 * ZG::P];
    __shared__ T sa[2 * AG::P];
    __shared__ T sk[AG::P];
    __shared__ T fx[4 * FXN];                 // K D_x z, columns x0-2 .. x0+33, rows of the tile
    __shared__ T fy[4 * FYN];                 // K D_y z, rows y0-2 .. y0+TY+1
    __shared__ double red[4];
    const int tx = threadIdx.x % kMTX, ty = threadIdx.x / kMTX;
    const int x0 = blockIdx.x * kMTX, y0 = blockIdx.y * TY;
    const int x = x0 + tx, y = y0 + ty;
    const int z0 = blockIdx.z * kZC, z1 = min(z0 + kZC, g.nz);
    const bool mine = x < g.nx && y < g.ny;
    const long long np = g.npts, nxy = (long long)g.nx * g.ny;
    const bool vper = g.bcv == JFNK_BC_PERIODIC;
    const T ihx = T(g.idx), ihy = T(g.idy), ihz = T(g.idz);
    const int cx = min(x, g.nx - 1), cy = min(y, g.ny - 1);   // own column (clamped: unused outside)
    const long long col = (long long)cy * g.nx + cx;
    // column value of field k of a state at plane zz (z reflection only)
    auto colv = [&](const T* __restrict__ a, int k, int zz) {
        int sz_;
        const int mz = map3(zz, g.nz, vper, sz_);
        const T v = a[(long long)k * np + mz * nxy + col];
        return odd3(k, 0, 0, sz_, g.bcv) ? -v : v;
    };
    // coefficient of flux slot f (0 u, 1 v, 2 w, 3 theta) along a horizontal (or the
    // vertical) axis from a frozen viscosity
    auto kof = [&](T nuv, int f, bool vertical) {
        const Coef<T> kc = pc_k3(g, nuv);
        return f == 3 ? (vertical ? kc.hv : kc.hh) : (vertical ? kc.mv : kc.mh);
    };
    // column queues
    T zq[5][7], wq[5], fq[4][5];
    auto flux_z = [&](int zc_) {             // K D_z z at plane zc_ from zq planes zc_-2 .. zc_+2
        const T nuv = nuext(g, nu, cx, cy, zc_);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int k = f < 3 ? f : 4;
            qpush(fq[f], kof(nuv, f, true) * d5(zq[k][2], zq[k][3], zq[k][5], zq[k][6], ihz));
        }
    };
#pragma unroll
    for (int it = 0; it < 10; ++it) {         // planes z0-6 .. z0+3; fluxes at z0-2 .. z0+1
        const int n = z0 - 6 + it;
#pragma unroll
        for (int k = 0; k < 5; ++k) qpush(zq[k], colv(zin, k, n));
        if (it >= 6) flux_z(n - 2);
        if (it >= 6) qpush(wq, colv(u, 2, n - 2));
    }
    // in-plane staging: fixed positions per thread, reflected offsets set once
    Stager<T, 5, TY, NTHR, 5, false, 4> stz;
    Stager<T, 2, TY, NTHR, 2, false, 2> sta;
    stz.init(g, x0 - 4, y0 - 4);
    sta.init(g, x0 - 2, y0 - 2);
    constexpr int KPOS = (AG::P + NTHR - 1) / NTHR;
    int koff[KPOS];
    const long long ex = g.nx + 4, ey = g.ny + 4;
#pragma unroll
    for (int p = 0; p < KPOS; ++p) {
        const int idx = min((int)threadIdx.x + p * NTHR, AG::P - 1);
        const int ly = idx / AG::SX, lx = idx - ly * AG::SX;
        const int xe = min(max(x0 - 2 + lx + 2, 0), (int)ex - 1), ye = min(max(y0 - 2 + ly + 2, 0), (int)ey - 1);
        koff[p] = ye * (int)ex + xe;
    }
    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        // column: iterate at z+4, w at z+2, flux K D_z z at z+2
#pragma unroll
        for (int k = 0; k < 5; ++k) qpush(zq[k], colv(zin, k, z + 4));
        qpush(wq, colv(u, 2, z + 2));
        flux_z(z + 2);
        // plane z
        stz.load(g, zin, zin, z);
        sta.load(g, u, u, z);
        T kv[KPOS];
#pragma unroll
        for (int p = 0; p < KPOS; ++p) kv[p] = nu[(long long)(z + 2) * ex * ey + koff[p]];
        stz.store(sz);
        sta.store(sa);
#pragma unroll
        for (int p = 0; p < KPOS; ++p) {
            const int idx = (int)threadIdx.x + p * NTHR;
            if (idx < AG::P) sk[idx] = kv[p];
        }
        __syncthreads();
        // in-plane fluxes
        for (int idx = threadIdx.x; idx < 4 * FXN; idx += NTHR) {
            const int f = idx / FXN, rr = idx - f * FXN;
            const int row = rr / AG::SX, c = rr - row * AG::SX;
            const T* zp = sz + (f < 3 ? f : 4) * ZG::P + (row + 4) * ZG::SX + c + 2;
            fx[idx] = kof(sk[(row + 2) * AG::SX + c], f, false) * d5(zp[-2], zp[-1], zp[1], zp[2], ihx);
        }
        for (int idx = threadIdx.x; idx < 4 * FYN; idx += NTHR) {
            const int f = idx / FYN, rr = idx - f * FYN;
            const int row = rr / kMTX, c = rr - row * kMTX;
            const T* zp = sz + (f < 3 ? f : 4) * ZG::P + (row + 2) * ZG::SX + c + 4;
            fy[idx] = kof(sk[row * AG::SX + c + 2], f, false) *
                      d5(zp[-2 * ZG::SX], zp[-ZG::SX], zp[ZG::SX], zp[2 * ZG::SX], ihy);
        }
        __syncthreads();
        if (mine) {
            const long long i = (long long)z * nxy + col;
            const Coef<T> kc0 = pc_k3(g, sk[(ty + 2) * AG::SX + tx + 2]);
            const T dmom = pc_diag3(g, kc0.mh, kc0.mv), dth = pc_diag3(g, kc0.hh, kc0.hv);
            const T* ua = sa + (ty + 2) * AG::SX + tx + 2;
            const T* va = ua + AG::P;
            const T a[3] = {ua[0], va[0], wq[2]};
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const T* zp = sz + k * ZG::P + (ty + 4) * ZG::SX + tx + 4;
                const T zc = zp[0];
                T diff = T(0), cv = T(0);
                if (k != 3) {
                    const int f = k < 3 ? k : 3;
                    const T* fxp = fx + f * FXN + ty * AG::SX + tx + 2;
                    const T* fyp = fy + f * FYN + (ty + 2) * kMTX + tx;
                    diff += d5(fxp[-2], fxp[-1], fxp[1], fxp[2], ihx);
                    diff += d5(fyp[-2 * kMTX], fyp[-kMTX], fyp[kMTX], fyp[2 * kMTX], ihy);
                    diff += d5(fq[f][0], fq[f][1], fq[f][3], fq[f][4], ihz);
                }
                if (g.convection) {
                    cv += T(0.5) * (d5(ua[-2] * zp[-2], ua[-1] * zp[-1], ua[1] * zp[1], ua[2] * zp[2], ihx) +
                                    a[0] * d5(zp[-2], zp[-1], zp[1], zp[2], ihx));
                    constexpr int AS = AG::SX, ZS = ZG::SX;
                    cv += T(0.5) * (d5(va[-2 * AS] * zp[-2 * ZS], va[-AS] * zp[-ZS], va[AS] * zp[ZS],
                                       va[2 * AS] * zp[2 * ZS], ihy) +
                                    a[1] * d5(zp[-2 * ZS], zp[-ZS], zp[ZS], zp[2 * ZS], ihy));
                    cv += T(0.5) * (d5(wq[0] * zq[k][0], wq[1] * zq[k][1], wq[3] * zq[k][3], wq[4] * zq[k][4], ihz) +
                                    a[2] * d5(zq[k][0], zq[k][1], zq[k][3], zq[k][4], ihz));
                }
                const T Pz = T(g.two_dt) * zc + (cv - diff);
                const T dd = k == 3 ? T(g.two_dt) : (k == 4 ? dth : dmom);
                const T zn = zc + (r[k * np + i] - Pz) / dd;
                zout[k * np + i] = zn;
                acc += (double)zn * (double)zn;
            }
        }
        __syncthreads();
    }
    if (ea.partials) {
        const double t = block_sum256(acc, red);
        if (threadIdx.x == 0) ea.partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
    }
}

// frozen eddy viscosity on the ring-2 extended grid
template <typename T>
__global__ __launch_bounds__(256) void k3_frozen_nu(Geo g, const T* __restrict__ u, T* __restrict__ nu) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    int x, y, z;
    if (!ext_point(g, i, x, y, z)) return;
    T S[6], th[3];
    strain3(g, u, x, y, z, S, th);
    T n, k;
    closure3(g, frob3(S, S), n, k);
    nu[i] = n;
}

// z0 = v / d (v = V_j / div written back); returns the thread's ||z||^2
template <typename T>
__global__ __launch_bounds__(256) void k3_pc_diag(Geo g, const T* __restrict__ nu, T* __restrict__ vj,
                                                  const double* __restrict__ div, T* __restrict__ z, EpsArgs ea) {
    __shared__ double red[4];
    // a grid-stride loop over points (32-bit indices: the launcher checks
    // npts < 2^31), so that the per-launch constants are formed once per thread
    // and the FD step's finishing block adds at most one partial sum per block
    const int np = (int)g.npts, nx = g.nx, nxy = g.nx * g.ny;
    const int ex = g.nx + 4, exy = (g.nx + 4) * (g.ny + 4);
    const double dv = div ? *div : 1.0;
    double acc = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < np; i += gridDim.x * 256) {
        const int zz = i / nxy, rem = i - zz * nxy, y = rem / nx, x = rem - y * nx;
        const Coef<T> kc = pc_k3(g, nu[(zz + 2) * exy + (y + 2) * ex + (x + 2)]);
        const T dm = pc_diag3(g, kc.mh, kc.mv), dt_ = pc_diag3(g, kc.hh, kc.hv);
        const T dd[5] = {dm, dm, dm, T(g.two_dt), dt_};
        T vv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) vv[k] = vj[(long long)k * np + i];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if (div) {
                vv[k] = (T)((double)vv[k] / dv);
                vj[(long long)k * np + i] = vv[k];
            }
            const T zv = vv[k] / dd[k];
            z[(long long)k * np + i] = zv;
            acc += (double)zv * (double)zv;
        }
    }
    if (ea.partials) partial_eps(ea, acc, red);
}

// ---------------------------------------------------------------------------
// Per-point 3D kernels for any stencil half-width W (W = 4: the 9-point
// derivative of order parameter p = 3, section 2.3).  The same operators as the
// z-marching kernels, with every neighbour a global load through the mirror
// mapping (reach 2W for the composite D(K D .) and D(tau(D u)) stencils): the
// derived quantities and the frozen viscosity live on the grid grown by a ring
// of W, [9][nz+2W][ny+2W][nx+2W] and [nz+2W][ny+2W][nx+2W].
// ---------------------------------------------------------------------------
template <int W> struct Dc;
template <> struct Dc<2> {
    static constexpr double c[2] = {2.0 / 3.0, -1.0 / 12.0};
    static constexpr double sumsq2 = 65.0 / 72.0;
};
template <> struct Dc<4> {
    static constexpr double c[4] = {272.0 / 365.0, -53.0 / 365.0, 16.0 / 1095.0, 1.0 / 2920.0};
    static constexpr double sumsq2 = 2.0 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + c[3] * c[3]);
};

// sum_m c_m (f(m) - f(-m)) ih for a tap functor f(offset)
template <int W, typename T, typename F>
__device__ __forceinline__ T dW(F f, T ih) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < W; ++m) acc += (T(Dc<W>::c[m]) * ih) * (f(m + 1) - f(-m - 1));
    return acc;
}

__device__ __forceinline__ double ihg(const Geo& g, int a) { return a == 0 ? g.idx : (a == 1 ? g.idy : g.idz); }

// derivative of state field f along axis a at (possibly ghost) (x, y, z)
template <int W, typename T>
__device__ __forceinline__ T dfW(const Geo& g, const T* __restrict__ u, int f, int a, int x, int y, int z) {
    const int ex = a == 0, ey = a == 1, ez = a == 2;
    return dW<W>([&](int o) { return ld(g, u, f, x + o * ex, y + o * ey, z + o * ez); }, T(ihg(g, a)));
}

// index on the grid grown by a ring of W
template <int W>
__device__ __forceinline__ long long extW(const Geo& g, int x, int y, int z) {
    return ((long long)(z + W) * (g.ny + 2 * W) + (y + W)) * (g.nx + 2 * W) + (x + W);
}
template <int W>
__device__ __forceinline__ long long next3W(const Geo& g) {
    return (long long)(g.nx + 2 * W) * (g.ny + 2 * W) * (g.nz + 2 * W);
}
template <int W>
__device__ __forceinline__ bool ext_pointW(const Geo& g, long long i, int& x, int& y, int& z) {
    const long long ex = g.nx + 2 * W, ey = g.ny + 2 * W, ez = g.nz + 2 * W;
    if (i >= ex * ey * ez) return false;
    x = (int)(i % ex) - W;
    y = (int)((i / ex) % ey) - W;
    z = (int)(i / (ex * ey)) - W;
    return true;
}

template <int W, typename T>
__device__ __forceinline__ void strainW(const Geo& g, const T* __restrict__ u, int x, int y, int z, T S[6], T th[3]) {
    T gr[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] = dfW<W>(g, u, i, j, x, y, z);
    S[0] = gr[0][0];
    S[1] = gr[1][1];
    S[2] = gr[2][2];
    S[3] = T(0.5) * (gr[0][1] + gr[1][0]);
    S[4] = T(0.5) * (gr[0][2] + gr[2][0]);
    S[5] = T(0.5) * (gr[1][2] + gr[2][1]);
#pragma unroll
    for (int j = 0; j < 3; ++j) th[j] = dfW<W>(g, u, 4, j, x, y, z);
}

// stress / heat flux (or, with PAIR, their stable FD differences) on the grid
// grown by W, one thread per point
template <int W, typename T, bool PAIR>
__global__ __launch_bounds__(256) void k3g_derived(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                   double eps_in, const double* __restrict__ eps_dev,
                                                   T* __restrict__ d) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    int x, y, z;
    if (!ext_pointW<W>(g, i, x, y, z)) return;
    const long long ne = next3W<W>(g);
    if (!PAIR) {
        T S[6], th[3];
        strainW<W>(g, u, x, y, z, S, th);
        const Coef<T> k = closure3c(g, frob3(S, S));
        const T third = (S[0] + S[1] + S[2]) * T(1.0 / 3.0);
#pragma unroll
        for (int c = 0; c < 6; ++c) d[c * ne + i] = T(2) * (vert3(c) ? k.mv : k.mh) * (c < 3 ? S[c] - third : S[c]);
#pragma unroll
        for (int j = 0; j < 3; ++j) d[(6 + j) * ne + i] = (j == 2 ? k.hv : k.hh) * th[j];
        return;
    }
    const T e = T(eps_dev ? *eps_dev : eps_in);
    T SU[6], SV[6], tU[3], tV[3], SW[6];
    strainW<W>(g, u, x, y, z, SU, tU);
    strainW<W>(g, v, x, y, z, SV, tV);
#pragma unroll
    for (int c = 0; c < 6; ++c) SW[c] = SU[c] + e * SV[c];
    const Coef<T> ka = closure3c(g, frob3(SU, SU));
    Coef<T> dk = {T(0), T(0), T(0), T(0)};
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
        const T den = sqrt(frob3(SU, SU)) + sqrt(frob3(SW, SW));
        const T num = T(2) * frob3(SU, SV) + e * frob3(SV, SV);
        if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
            const T dnu = den > T(0) ? T(g.smag) * T(1.4142135623730951) * num / den : T(0);
            dk = {dnu, dnu, dnu * T(g.inv_pr), dnu * T(g.inv_pr)};
        } else {
            dk = deardorff_diff(g, T(sqrt(frob3(SU, SU))), den > T(0) ? num / den : T(0), e);
        }
    }
    const T trw = (SW[0] + SW[1] + SW[2]) * T(1.0 / 3.0), trv = (SV[0] + SV[1] + SV[2]) * T(1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const T dw = c < 3 ? SW[c] - trw : SW[c];
        const T dv = c < 3 ? SV[c] - trv : SV[c];
        d[c * ne + i] = T(2) * (vert3(c) ? dk.mv : dk.mh) * dw + T(2) * (vert3(c) ? ka.mv : ka.mh) * dv;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
        d[(6 + j) * ne + i] = (j == 2 ? dk.hv : dk.hh) * (tU[j] + e * tV[j]) + (j == 2 ? ka.hv : ka.hh) * tV[j];
}

// the operator per grid point: MODE 0 out = F (what 0), 2u/dt + F (1),
// 2u/dt - F - f (2); MODE 1 Jv = 2v/dt - [F(u + e v) - F(u)]/e expanded
template <int W, typename T, int MODE>
__global__ __launch_bounds__(256) void k3g_point(Geo g, const T* __restrict__ u, const T* __restrict__ v,
                                                 double eps_in, const double* __restrict__ eps_dev,
                                                 const T* __restrict__ d, const T* __restrict__ f,
                                                 T* __restrict__ out, int what) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.npts) return;
    const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
    const long long np = g.npts, ne = next3W<W>(g);
    const T e = MODE == 1 ? T(eps_dev ? *eps_dev : eps_in) : T(0);
    const T th0 = T(g.theta0);
    const T* pb = Bg<T>::pbar(g);
    const T* dpb = Bg<T>::dpbar(g);
    // divergence of derived component c along axis j
    auto dd = [&](int c, int j) -> T {
        const int ex = j == 0, ey = j == 1, ez = j == 2;
        return dW<W>([&](int o) { return d[c * ne + extW<W>(g, x + o * ex, y + o * ey, z + o * ez)]; },
                     T(ihg(g, j)));
    };
    T A[5], B[5], dF[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        A[k] = u[k * np + i];
        B[k] = MODE == 1 ? v[k * np + i] : T(0);
    }
    T divA = T(0), divB = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int ex = j == 0, ey = j == 1, ez = j == 2;
        const T ih = T(ihg(g, j));
        for (int k = 0; k < 5; ++k) {
            auto a = [&](int o) { return ld(g, u, k, x + o * ex, y + o * ey, z + o * ez); };
            auto aj = [&](int o) { return ld(g, u, j, x + o * ex, y + o * ey, z + o * ez); };
            if (MODE == 0) {
                if (g.convection) {
                    const T flux = dW<W>([&](int o) { return aj(o) * a(o); }, ih);
                    dF[k] -= T(0.5) * (flux + A[j] * dW<W>(a, ih));
                }
                if (k == j) divA += dW<W>(a, ih);
            } else {
                auto b = [&](int o) { return ld(g, v, k, x + o * ex, y + o * ey, z + o * ez); };
                auto bj = [&](int o) { return ld(g, v, j, x + o * ex, y + o * ey, z + o * ez); };
                const T dA = dW<W>(a, ih), dB = dW<W>(b, ih);
                if (g.convection) {
                    const T flux = dW<W>([&](int o) { return aj(o) * b(o) + bj(o) * (a(o) + e * b(o)); }, ih);
                    dF[k] -= T(0.5) * (flux + A[j] * dB + B[j] * (dA + e * dB));
                }
                if (k == j) {
                    divA += dA;
                    divB += dB;
                }
            }
        }
    }
    const T* P = MODE == 1 ? v : u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dF[c] -= th0 * dfW<W>(g, P, 3, c, x, y, z);
#pragma unroll
        for (int j = 0; j < 3; ++j) dF[c] += dd(tix(c, j), j);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) dF[4] += dd(6 + j, j);
    if (MODE == 0) {
        dF[2] += T(g.g_theta0) * A[4];
        if (g.energy_test)
            dF[3] -= T(g.kappa_cp) * divA;
        else
            dF[3] -= A[2] * dpb[z] + T(g.kappa) * (pb[z] + A[3]) * divA;
        dF[4] -= T(g.beta) * A[2];
        if (z == 0 && !g.energy_test) dF[4] += Bg<T>::sflux(g)[(long long)y * g.nx + x];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            T r;
            if (what == 0) r = dF[k];
            else if (what == 1) r = T(g.two_dt) * A[k] + dF[k];
            else r = T(g.two_dt) * A[k] - dF[k] - (f ? f[k * np + i] : T(0));
            out[k * np + i] = r;
        }
    } else {
        dF[2] += T(g.g_theta0) * B[4];
        if (g.energy_test)
            dF[3] -= T(g.kappa_cp) * divB;
        else
            dF[3] -= B[2] * dpb[z] + T(g.kappa) * ((pb[z] + A[3]) * divB + B[3] * divA + e * B[3] * divB);
        dF[4] -= T(g.beta) * B[2];
#pragma unroll
        for (int k = 0; k < 5; ++k) out[k * np + i] = T(g.two_dt) * B[k] - dF[k];
    }
}

// frozen eddy viscosity on the grid grown by W
template <int W, typename T>
__global__ __launch_bounds__(256) void k3g_frozen_nu(Geo g, const T* __restrict__ u, T* __restrict__ nu) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    int x, y, z;
    if (!ext_pointW<W>(g, i, x, y, z)) return;
    T S[6], th[3];
    strainW<W>(g, u, x, y, z, S, th);
    T n, k;
    closure3(g, frob3(S, S), n, k);
    nu[i] = n;
}

template <int W, typename T>
__device__ __forceinline__ T pc_diagW(const Geo& g, T kh, T kv) {
    const T cD = T(Dc<W>::sumsq2);
    if (g.closure == JFNK_CLOSURE_DEARDORFF)
        return T(g.two_dt) + cD * (kh * T(g.idx * g.idx + g.idy * g.idy) + kv * T(g.idz * g.idz));
    return T(g.two_dt) + cD * kh * T(g.idx * g.idx + g.idy * g.idy + g.idz * g.idz);
}

// z0 = v / d (v = V_j / div written back); the thread's ||z||^2 to the partials
template <int W, typename T>
__global__ __launch_bounds__(256) void k3g_pc_diag(Geo g, const T* __restrict__ nu, T* __restrict__ vj,
                                                   const double* __restrict__ div, T* __restrict__ z, EpsArgs ea) {
    __shared__ double red[4];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double acc = 0.0;
    if (i < g.npts) {
        const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), zz = (int)(i / ((long long)g.nx * g.ny));
        const Coef<T> kc = pc_k3(g, nu[extW<W>(g, x, y, zz)]);
        const T dm = pc_diagW<W>(g, kc.mh, kc.mv), dt_ = pc_diagW<W>(g, kc.hh, kc.hv);
        const T dg[5] = {dm, dm, dm, T(g.two_dt), dt_};
        const double dv = div ? *div : 1.0;
        const long long np = g.npts;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            T vv = vj[k * np + i];
            if (div) {
                vv = (T)((double)vv / dv);
                vj[k * np + i] = vv;
            }
            const T zv = vv / dg[k];
            z[k * np + i] = zv;
            acc += (double)zv * (double)zv;
        }
    }
    if (ea.partials) partial_eps(ea, acc, red);
}

// one Jacobi sweep of the field-block preconditioner, one thread per point:
// zout = zin + (r - P zin)/d with P z = (2/dt) z + C(a(u); z) - sum_j D_j(K D_j z)
template <int W, typename T>
__global__ __launch_bounds__(256) void k3g_pc_sweep(Geo g, const T* __restrict__ u, const T* __restrict__ nu,
                                                    const T* __restrict__ r, const T* __restrict__ zin,
                                                    T* __restrict__ zout, EpsArgs ea) {
    __shared__ double red[4];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double acc = 0.0;
    if (i < g.npts) {
        const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
        const long long np = g.npts;
        const Coef<T> kc0 = pc_k3(g, nu[extW<W>(g, x, y, z)]);
        const T dmom = pc_diagW<W>(g, kc0.mh, kc0.mv), dth = pc_diagW<W>(g, kc0.hh, kc0.hv);
        for (int k = 0; k < 5; ++k) {
            const T zc = zin[k * np + i];
            T t = T(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ex = j == 0, ey = j == 1, ez = j == 2;
                const T ih = T(ihg(g, j));
                auto zz = [&](int o) { return ld(g, zin, k, x + o * ex, y + o * ey, z + o * ez); };
                if (k != 3) {
                    // D_j (K D_j z): K frozen on the grid grown by W
                    auto flux = [&](int o) {
                        const int xo = x + o * ex, yo = y + o * ey, zo = z + o * ez;
                        const Coef<T> kc = pc_k3(g, nu[extW<W>(g, xo, yo, zo)]);
                        const T K = k == 4 ? (j == 2 ? kc.hv : kc.hh) : (j == 2 ? kc.mv : kc.mh);
                        return K * dW<W>([&](int q) { return ld(g, zin, k, xo + q * ex, yo + q * ey, zo + q * ez); },
                                         ih);
                    };
                    t -= dW<W>(flux, ih);
                }
                if (g.convection) {
                    auto aj = [&](int o) { return ld(g, u, j, x + o * ex, y + o * ey, z + o * ez); };
                    t += T(0.5) * (dW<W>([&](int o) { return aj(o) * zz(o); }, ih) + u[j * np + i] * dW<W>(zz, ih));
                }
            }
            const T Pz = T(g.two_dt) * zc + t;
            const T dd = k == 3 ? T(g.two_dt) : (k == 4 ? dth : dmom);
            const T zn = zc + (r[k * np + i] - Pz) / dd;
            zout[k * np + i] = zn;
            acc += (double)zn * (double)zn;
        }
    }
    if (ea.partials) partial_eps(ea, acc, red);
}

inline int blocks(long long n) { return (int)((n + 255) / 256); }
inline long long next3(const Geo& g) { return (long long)(g.nx + 4) * (g.ny + 4) * (g.nz + 4); }

}  // namespace

inline dim3 march_grid(int nx, int ny, int nz, int ty) {
    return dim3((nx + kMTX - 1) / kMTX, (ny + ty - 1) / ty, (nz + kZC - 1) / kZC);
}

template <int W>
inline long long next3W_host(const Geo& g) {
    return (long long)(g.nx + 2 * W) * (g.ny + 2 * W) * (g.nz + 2 * W);
}

template <typename T>
hipError_t launch3_apply_F(const Geo& g, const T* u, const T* f, T* out, int what, T* dbuf, hipStream_t s) {
    if (g.W == 4) {
        hipLaunchKernelGGL((k3g_derived<4, T, false>), dim3(blocks(next3W_host<4>(g))), dim3(256), 0, s, g, u,
                           (const T*)nullptr, 0.0, (const double*)nullptr, dbuf);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k3g_point<4, T, 0>), dim3(blocks(g.npts)), dim3(256), 0, s, g, u, (const T*)nullptr, 0.0,
                           (const double*)nullptr, (const T*)dbuf, f, out, what);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k3m_derived<T, false>), march_grid(g.nx + 4, g.ny + 4, g.nz + 4, 8), dim3(256), 0, s, g, u,
                       (const T*)nullptr, 0.0, (const double*)nullptr, dbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k3m_point<T, 0, 8>), march_grid(g.nx, g.ny, g.nz, 8), dim3(256), 0, s, g, u,
                       (const T*)nullptr, 0.0, (const double*)nullptr, (const T*)dbuf, f, out, what);
    return hipGetLastError();
}

// Planes per workgroup of the single-pass Jv: enough z chunks for one
// workgroup per compute unit (256 CUs; a workgroup of 32 x 16 columns holds
// 157 KB of LDS), at least 16 planes per chunk (each chunk re-forms four
// planes of derived quantities at its start).
inline int fused_kzc(int nx, int ny, int nz, int ty) {
    const long long cols = (long long)((nx + 31) / 32) * ((ny + ty - 1) / ty);
    const long long want = (256 + cols - 1) / cols;
    int kzc = (int)((nz + want - 1) / want);
    kzc = std::max(kzc, std::min(nz, 16));
    return std::max(1, kzc);
}

hipError_t launch3_jv_fused(const Geo& g, const float* u, const float* v, double eps, const double* eps_dev,
                            float* out, hipStream_t s) {
    constexpr int TY = 16;
    const int kzc = fused_kzc(g.nx, g.ny, g.nz, TY);
    const int nblk = ((g.nx + 31) / 32) * ((g.ny + TY - 1) / TY) * ((g.nz + kzc - 1) / kzc);
    hipLaunchKernelGGL((k3f_jv<TY>), dim3(nblk), dim3(32 * TY + 256), 0, s, g, u, v, eps, eps_dev, out, kzc);
    return hipGetLastError();
}

// FP64 Jv points use 32 x 4 columns (LDS)
template <typename T>
hipError_t launch3_jv(const Geo& g, const T* u, const T* v, double eps, const double* eps_dev, T* out, T* dbuf,
                      hipStream_t s) {
    if (g.W == 4) {
        hipLaunchKernelGGL((k3g_derived<4, T, true>), dim3(blocks(next3W_host<4>(g))), dim3(256), 0, s, g, u, v, eps,
                           eps_dev, dbuf);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k3g_point<4, T, 1>), dim3(blocks(g.npts)), dim3(256), 0, s, g, u, v, eps, eps_dev,
                           (const T*)dbuf, (const T*)nullptr, out, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k3m_derived<T, true>), march_grid(g.nx + 4, g.ny + 4, g.nz + 4, 8), dim3(256), 0, s, g, u, v,
                       eps, eps_dev, dbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL((k3m_point<T, 1, 4>), march_grid(g.nx, g.ny, g.nz, 4), dim3(128), 0, s, g, u, v, eps,
                           eps_dev, (const T*)dbuf, (const T*)nullptr, out, 0);
    else
        hipLaunchKernelGGL((k3m_point<T, 1, 8>), march_grid(g.nx, g.ny, g.nz, 8), dim3(256), 0, s, g, u, v, eps,
                           eps_dev, (const T*)dbuf, (const T*)nullptr, out, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_frozen_nu(const Geo& g, const T* u, T* nu, hipStream_t s) {
    if (g.W == 4) {
        hipLaunchKernelGGL((k3g_frozen_nu<4, T>), dim3(blocks(next3W_host<4>(g))), dim3(256), 0, s, g, u, nu);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k3_frozen_nu<T>), dim3(blocks(next3(g))), dim3(256), 0, s, g, u, nu);
    return hipGetLastError();
}

// blocks of the 3D preconditioner diagonal (grid-stride): eight per CU
constexpr int kPcDiagBlocks = 2048;

template <typename T>
hipError_t launch3_pc_diag(const Geo& g, const T* nu, T* vj, const double* div, T* z, const EpsArgs& ea,
                           hipStream_t s) {
    int nb = blocks(g.npts);
    if (g.W == 4) {
        hipLaunchKernelGGL((k3g_pc_diag<4, T>), dim3(nb), dim3(256), 0, s, g, nu, vj, div, z, ea);
    } else {
        if (g.npts >= (1LL << 31) || (long long)(g.nx + 4) * (g.ny + 4) * (g.nz + 4) >= (1LL << 31))
            return hipErrorInvalidValue;
        nb = nb < kPcDiagBlocks ? nb : kPcDiagBlocks;
        hipLaunchKernelGGL((k3_pc_diag<T>), dim3(nb), dim3(256), 0, s, g, nu, vj, div, z, ea);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    return launch_eps_finish(nb, ea, s);
}

template <typename T>
hipError_t launch3_pc_sweep(const Geo& g, const T* u, const T* nu, const T* r, const T* zin, T* zout,
                            const EpsArgs& ea, hipStream_t s) {
    if (g.W == 4) {
        const int nb = blocks(g.npts);
        hipLaunchKernelGGL((k3g_pc_sweep<4, T>), dim3(nb), dim3(256), 0, s, g, u, nu, r, zin, zout, ea);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !ea.partials) return e;
        return launch_eps_finish(nb, ea, s);
    }
    const dim3 grid = march_grid(g.nx, g.ny, g.nz, 8);
    hipLaunchKernelGGL((k3m_pc_sweep<T>), grid, dim3(256), 0, s, g, u, nu, r, zin, zout, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ea.partials) return e;
    return launch_eps_finish((int)(grid.x * grid.y * grid.z), ea, s);
}

#define JFNK_INST3(T)                                                                                          \
    template hipError_t launch3_apply_F<T>(const Geo&, const T*, const T*, T*, int, T*, hipStream_t);          \
    template hipError_t launch3_jv<T>(const Geo&, const T*, const T*, double, const double*, T*, T*,            \
                                      hipStream_t);                                                            \
    template hipError_t launch3_frozen_nu<T>(const Geo&, const T*, T*, hipStream_t);                           \
    template hipError_t launch3_pc_diag<T>(const Geo&, const T*, T*, const double*, T*, const EpsArgs&,        \
                                           hipStream_t);                                                       \
    template hipError_t launch3_pc_sweep<T>(const Geo&, const T*, const T*, const T*, const T*, T*,             \
                                            const EpsArgs&, hipStream_t);
JFNK_INST3(double)
JFNK_INST3(float)
#undef JFNK_INST3

}  // namespace jfnk
