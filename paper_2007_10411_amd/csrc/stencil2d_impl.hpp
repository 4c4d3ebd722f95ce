// Device bodies of the 2D stencil kernels of the JFNK hot path for gfx950
// (shared by the single-grid kernels and the batched ensemble kernels).
//
// Discretisation (sections 2.1-2.4 of the paper, equations 1-5 and 9):
//   D      Deslauriers-Dubuc collocation derivative of order 2p with half-width W:
//          (D a)_i = sum_{m=1..W} c_m (a_{i+m} - a_{i-m}) / h, p = 2 (W = 2, 5 points):
//          c = 2/3, -1/12; p = 3 (W = 4, 9 points): c = 272/365, -53/365, 16/1095,
//          1/2920
//   C      skew-symmetric convection 1/2 sum_j [ D_j(a_j phi) + a_j D_j phi ]
//   tau    2 nu (S - tr(S)/3 I), S = sym(grad u), nu = (cs Delta)^2 sqrt(2 S:S)
//   q      (nu / Pr_t) D theta
//   F_u_i  = -C(u; u_i) - theta0 D_i p + delta_iz (g/theta0) theta + D_j tau_ij
//   F_p    = -C(u; p) - w dp_bar/dz - kappa (p_bar + p) div u
//   F_th   = -C(u; theta) - beta w + D_j q_j + [k = 0] Q / dz
// Walls sit on the cell faces; fields are extended by mirror reflection with a
// parity (normal velocity odd, tangential velocity odd at a no-slip bottom,
// everything else even) or periodically.  The composite D(tau(D u)) reaches 2W
// points, so every tile stages its primitives with a halo of 2W in LDS, forms
// the stress and heat flux on a ring of W and differentiates those.  W is a
// template parameter of every tile body (default 2).
//
// Tile: TX x TZ output points per 256-thread workgroup, x fastest so that each
// wavefront reads 64 consecutive points of a row (coalesced).

#pragma once

#include "jfnk_internal.hpp"
#include "reduce.hpp"
#include "exchange.hpp"

namespace jfnk {
namespace s2d {


constexpr int kHalo = 4;

// Source index of extended position e along an axis of n points, and which
// ghost side it came from (0 interior, 1 low, 2 high).  Positions further out
// than the halo are clamped (they only feed outputs outside the domain).
__device__ __forceinline__ int map_axis(int e, int n, bool periodic, int& side) {
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

// Reflection sign of 2D field f (0 u, 1 w, 2 p, 3 theta).
__device__ __forceinline__ int sign2d(int f, int sx, int sz, int bcv) {
    int s = 1;
    if (sx && f == 0) s = -s;
    if (sz) {
        if (f == 1) s = -s;
        else if (f == 0 && bcv == JFNK_BC_NO_SLIP_BOTTOM && sz == 1) s = -s;
    }
    return s;
}

template <typename T>
__device__ __forceinline__ T d5(T m2, T m1, T p1, T p2, T ih) {
    // weights scaled by 1/h once (shared by every derivative along the axis)
    return (T(2.0 / 3.0) * ih) * (p1 - m1) - (T(1.0 / 12.0) * ih) * (p2 - m2);
}

// One-sided weights c_m of the derivative of half-width W, and 2 sum_m c_m^2
// (the diagonal of D(K D .) per unit K / h^2).
template <int W> struct DW;
template <> struct DW<2> {
    static constexpr double c[2] = {2.0 / 3.0, -1.0 / 12.0};
    static constexpr double sumsq2 = 65.0 / 72.0;
};
template <> struct DW<4> {
    static constexpr double c[4] = {272.0 / 365.0, -53.0 / 365.0, 16.0 / 1095.0, 1.0 / 2920.0};
    static constexpr double sumsq2 = 2.0 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + c[3] * c[3]);
};

// sum_m c_m (f(m) - f(-m)) * ih for a tap functor f(offset)
template <int W, typename T, typename F>
__device__ __forceinline__ T dtaps(F f, T ih) {
    if constexpr (W == 2) {
        return d5(f(-2), f(-1), f(1), f(2), ih);
    } else {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < W; ++m) acc += (T(DW<W>::c[m]) * ih) * (f(m + 1) - f(-m - 1));
        return acc;
    }
}

// x- and z-derivative of an LDS array at (z, x) with row stride S
template <typename T, int S, int W = 2>
__device__ __forceinline__ T dx_s(const T* a, int z, int x, T ih) {
    const T* r = a + z * S + x;
    return dtaps<W>([&](int o) { return r[o]; }, ih);
}
template <typename T, int S, int W = 2>
__device__ __forceinline__ T dz_s(const T* a, int z, int x, T ih) {
    const T* r = a + z * S + x;
    return dtaps<W>([&](int o) { return r[o * S]; }, ih);
}

// Derivatives of a product a*b stored in two LDS arrays
template <typename T, int S, int W = 2>
__device__ __forceinline__ T dx_prod(const T* a, const T* b, int z, int x, T ih) {
    const T* ra = a + z * S + x;
    const T* rb = b + z * S + x;
    return dtaps<W>([&](int o) { return ra[o] * rb[o]; }, ih);
}
template <typename T, int S, int W = 2>
__device__ __forceinline__ T dz_prod(const T* a, const T* b, int z, int x, T ih) {
    const T* ra = a + z * S + x;
    const T* rb = b + z * S + x;
    return dtaps<W>([&](int o) { return ra[o * S] * rb[o * S]; }, ih);
}

// Threads per tile workgroup (every tile kernel is launched with this many).
constexpr int kTileThreads = 256;

// Copy of the n-field state (field stride np) with halo H, held in registers
// between load() and store(): load() issues all global loads of the tile (the
// reflected ghosts by the parity mapping) before any LDS store, so their
// latencies overlap; store() writes LDS s[f][SZ][SX].
template <typename T, int TX, int TZ, int NFL, int H>
struct TileStage {
    static constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H, N = SZ * SX;
    static constexpr int IT = (N + kTileThreads - 1) / kTileThreads;
    static constexpr int NW = (IT * NFL + 31) / 32;
    T r[IT][NFL];
    unsigned neg[NW];   // sign bits, bit (it NFL + f)
    __device__ __forceinline__ void load(const Geo& g, const T* __restrict__ u, int x0, int z0, int f_first) {
        const long long np = g.npts;
#pragma unroll
        for (int w = 0; w < NW; ++w) neg[w] = 0u;
        if (x0 >= H && z0 >= H && x0 + TX + H <= g.nx && z0 + TZ + H <= g.nz) {
            // the tile and its halo lie inside the grid: no wrap, no reflection
            const long long base = (long long)(z0 - H) * g.nx + (x0 - H);
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int idx = min((int)threadIdx.x + it * kTileThreads, N - 1);
                const int lz = idx / SX, lx = idx - lz * SX;
                const long long off = base + (long long)lz * g.nx + lx;
#pragma unroll
                for (int f = 0; f < NFL; ++f) r[it][f] = u[(long long)(f_first + f) * np + off];
            }
            return;
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = min((int)threadIdx.x + it * kTileThreads, N - 1);
            const int lz = idx / SX, lx = idx - lz * SX;
            int sx, sz;
            const int gx = map_axis(x0 + lx - H, g.nx, g.bcl == JFNK_BC_PERIODIC, sx);
            const int gz = map_axis(z0 + lz - H, g.nz, g.bcv == JFNK_BC_PERIODIC, sz);
            const long long off = (long long)gz * g.nx + gx;
#pragma unroll
            for (int f = 0; f < NFL; ++f) {
                r[it][f] = u[(long long)(f_first + f) * np + off];
                const int b = it * NFL + f;
                if (sign2d(f_first + f, sx, sz, g.bcv) < 0) neg[b / 32] |= 1u << (b % 32);
            }
        }
    }
    __device__ __forceinline__ void store(T* s) const {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = (int)threadIdx.x + it * kTileThreads;
            if (idx < N) {
#pragma unroll
                for (int f = 0; f < NFL; ++f) {
                    const int b = it * NFL + f;
                    s[f * N + idx] = (neg[b / 32] >> (b % 32)) & 1u ? -r[it][f] : r[it][f];
                }
            }
        }
    }
    // this state plus e times state o, staged at the same positions (the same
    // fields, so the same reflection signs)
    __device__ __forceinline__ void store_sum(T* s, const TileStage& o, T e) const {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = (int)threadIdx.x + it * kTileThreads;
            if (idx < N) {
#pragma unroll
                for (int f = 0; f < NFL; ++f) {
                    const int b = it * NFL + f;
                    const T v = r[it][f] + e * o.r[it][f];
                    s[f * N + idx] = (neg[b / 32] >> (b % 32)) & 1u ? -v : v;
                }
            }
        }
    }
};

// Stage the n-field state (field stride np) with halo H into LDS s[f][SZ][SX].
template <typename T, int TX, int TZ, int NFL, int H = kHalo>
__device__ __forceinline__ void stage_fields(const Geo& g, const T* __restrict__ u, T* s, int x0, int z0,
                                             int f_first) {
    TileStage<T, TX, TZ, NFL, H> st;
    st.load(g, u, x0, z0, f_first);
    st.store(s);
}

// Isotropic coefficients (nu, K_theta) of S:S = s2; for the anisotropic closure
// nu is the Smagorinsky viscosity from which its coefficients derive.
template <typename T>
__device__ __forceinline__ void closure_coeffs(const Geo& g, T s2, T& nu, T& kth) {
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

template <typename T>
__device__ __forceinline__ Coef<T> closure_coef(const Geo& g, T s2) {
    if (g.closure == JFNK_CLOSURE_DEARDORFF) return deardorff_coef(g, T(sqrt(s2)));
    T nu, kth;
    closure_coeffs(g, s2, nu, kth);
    return {nu, nu, kth, kth};
}

// ---------------------------------------------------------------------------
// Point bodies of F and Jv over LDS accessors.  An accessor returns field f at
// row offset oz and column offset ox from the point; the tile kernels read
// contiguous rows, the row-marching kernels rows held in the slots of a ring.
// ---------------------------------------------------------------------------
template <typename T, int FS, int RS>
struct TileAcc {      // rows contiguous with stride RS, fields FS apart
    const T* p;       // field 0 at the point
    __device__ __forceinline__ T at(int f, int oz, int ox) const { return p[f * FS + oz * RS + ox]; }
};
template <typename T, int FS, int W>
struct RingAcc {      // rows z-W..z+W in ring slots, fields FS apart
    const T* r[2 * W + 1];   // field 0 of each row at the point's column
    __device__ __forceinline__ T at(int f, int oz, int ox) const { return r[oz + W][f * FS + ox]; }
};

template <int W, typename T, typename A>
__device__ __forceinline__ T acc_dx(const A& a, int f, T ih) {
    return dtaps<W>([&](int o) { return a.at(f, 0, o); }, ih);
}
template <int W, typename T, typename A>
__device__ __forceinline__ T acc_dz(const A& a, int f, T ih) {
    return dtaps<W>([&](int o) { return a.at(f, o, 0); }, ih);
}

// Stress and heat flux (txx, txz, tzz, qx, qz) of the state held in P
// (fields u 0, w 1, theta 3).
template <int W, typename T, typename A>
__device__ __forceinline__ void derived_F_pt(const Geo& g, const A& P, T ihx, T ihz, T d[5]) {
    const T ux = acc_dx<W>(P, 0, ihx), uz = acc_dz<W>(P, 0, ihz);
    const T wx = acc_dx<W>(P, 1, ihx), wz = acc_dz<W>(P, 1, ihz);
    const T tx = acc_dx<W>(P, 3, ihx), tz = acc_dz<W>(P, 3, ihz);
    const T sxz = T(0.5) * (uz + wx);
    const T div = ux + wz;
    const T s2 = ux * ux + wz * wz + T(2) * sxz * sxz;
    const Coef<T> k = closure_coef(g, s2);
    const T third = div * T(1.0 / 3.0);
    d[0] = T(2) * k.mh * (ux - third);
    d[1] = T(2) * k.mv * sxz;
    d[2] = T(2) * k.mv * (wz - third);
    d[3] = k.hh * tx;
    d[4] = k.hv * tz;
}

// F at a point from the primitives P and the derived quantities D (txx 0,
// txz 1, tzz 2, qx 3, qz 4) at grid row gz.
template <int W, typename T, typename A, typename AD>
__device__ __forceinline__ void point_F_pt(const Geo& g, const A& P, const AD& D, int gz, T ihx, T ihz, T Fv[4]) {
    const T* pb = Bg<T>::pbar(g);
    const T* dpb = Bg<T>::dpbar(g);
    const T uu = P.at(0, 0, 0), ww = P.at(1, 0, 0), pp = P.at(2, 0, 0), th = P.at(3, 0, 0);
    const T ux = acc_dx<W>(P, 0, ihx), wz = acc_dz<W>(P, 1, ihz);
    const T div = ux + wz;
    T cu = 0, cw = 0, cp = 0, ct = 0;
    if (g.convection) {
        const T uz = acc_dz<W>(P, 0, ihz), wx = acc_dx<W>(P, 1, ihx);
        const T px = acc_dx<W>(P, 2, ihx), pz = acc_dz<W>(P, 2, ihz);
        const T tx = acc_dx<W>(P, 3, ihx), tz = acc_dz<W>(P, 3, ihz);
        auto dxp = [&](int fa, int fb) { return dtaps<W>([&](int o) { return P.at(fa, 0, o) * P.at(fb, 0, o); }, ihx); };
        auto dzp = [&](int fa, int fb) { return dtaps<W>([&](int o) { return P.at(fa, o, 0) * P.at(fb, o, 0); }, ihz); };
        cu = T(0.5) * (dxp(0, 0) + dzp(1, 0) + uu * ux + ww * uz);
        cw = T(0.5) * (dxp(0, 1) + dzp(1, 1) + uu * wx + ww * wz);
        cp = T(0.5) * (dxp(0, 2) + dzp(1, 2) + uu * px + ww * pz);
        ct = T(0.5) * (dxp(0, 3) + dzp(1, 3) + uu * tx + ww * tz);
    }
    const T th0 = T(g.theta0);
    Fv[0] = -th0 * acc_dx<W>(P, 2, ihx) + acc_dx<W>(D, 0, ihx) + acc_dz<W>(D, 1, ihz) - cu;
    Fv[1] = -th0 * acc_dz<W>(P, 2, ihz) + acc_dx<W>(D, 1, ihx) + acc_dz<W>(D, 2, ihz) - cw + T(g.g_theta0) * th;
    if (g.energy_test)
        Fv[2] = -cp - T(g.kappa_cp) * div;
    else
        Fv[2] = -cp - ww * dpb[gz] - T(g.kappa) * (pb[gz] + pp) * div;
    Fv[3] = acc_dx<W>(D, 3, ihx) + acc_dz<W>(D, 4, ihz) - ct - T(g.beta) * ww;
}

// Jv (stable finite-difference form):
//   [B(a + e b, c + e d) - B(a, c)] / e = B(a, d) + B(b, c) + e B(b, d)
//   nu difference: (cs Delta)^2 sqrt2 (2 S:T + e T:T) / (|S + e T| + |S|)
// The pair is staged as PW = u + e v and PB = v: derivatives of u + e v are taken
// directly, those of u as D(u + e v) - e Dv (the derivative is linear).
// Derived differences of the pair.
template <int W, typename T, typename A>
__device__ __forceinline__ void derived_jv_pt(const Geo& g, const A& PW, const A& PB, T e, T ihx, T ihz, T d[5]) {
    const T uxw = acc_dx<W>(PW, 0, ihx), uzw = acc_dz<W>(PW, 0, ihz);
    const T wxw = acc_dx<W>(PW, 1, ihx), wzw = acc_dz<W>(PW, 1, ihz);
    const T uxb = acc_dx<W>(PB, 0, ihx), uzb = acc_dz<W>(PB, 0, ihz);
    const T wxb = acc_dx<W>(PB, 1, ihx), wzb = acc_dz<W>(PB, 1, ihz);
    const T txw = acc_dx<W>(PW, 3, ihx), tzw = acc_dz<W>(PW, 3, ihz);
    const T txb = acc_dx<W>(PB, 3, ihx), tzb = acc_dz<W>(PB, 3, ihz);
    // strain of u + e v (c) and of v (b), then of u (a)
    const T cxx = uxw, czz = wzw, cxz = T(0.5) * (uzw + wxw);
    const T bxx = uxb, bzz = wzb, bxz = T(0.5) * (uzb + wxb);
    const T axx = cxx - e * bxx, azz = czz - e * bzz, axz = cxz - e * bxz;
    const T s2a = axx * axx + azz * azz + T(2) * axz * axz;
    Coef<T> ka, dk = {T(0), T(0), T(0), T(0)};
    if constexpr (std::is_same<T, float>::value) {
        // FP32: hardware square root and reciprocal (1 ulp, well inside the FP32
        // parity bar), |S(u)| shared by nu(u) and the nu difference
        if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
            const float sab = axx * bxx + azz * bzz + 2.f * axz * bxz;
            const float sbb = bxx * bxx + bzz * bzz + 2.f * bxz * bxz;
            const float s2c = cxx * cxx + czz * czz + 2.f * cxz * cxz;
            const float ma = __builtin_amdgcn_sqrtf(s2a);
            const float den = ma + __builtin_amdgcn_sqrtf(s2c);
            const float num = 2.f * sab + e * sbb;
            if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
                const float c = g.f.smag_s2, ip = g.f.inv_pr;
                const float nu = c * ma, dnu = den > 0.f ? c * num * __builtin_amdgcn_rcpf(den) : 0.f;
                ka = {nu, nu, nu * ip, nu * ip};
                dk = {dnu, dnu, dnu * ip, dnu * ip};
            } else {
                ka = deardorff_coef(g, ma);
                dk = deardorff_diff(g, ma, den > 0.f ? num / den : 0.f, e);
            }
        } else {
            ka = closure_coef(g, s2a);
        }
    } else {
        ka = closure_coef(g, s2a);
        if (g.closure == JFNK_CLOSURE_SMAGORINSKY || g.closure == JFNK_CLOSURE_DEARDORFF) {
            const T sab = axx * bxx + azz * bzz + T(2) * axz * bxz;
            const T sbb = bxx * bxx + bzz * bzz + T(2) * bxz * bxz;
            const T s2c = cxx * cxx + czz * czz + T(2) * cxz * cxz;
            const T den = sqrt(s2a) + sqrt(s2c);
            const T num = T(2) * sab + e * sbb;
            if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
                const T dnu = den > T(0) ? T(g.smag) * T(1.4142135623730951) * num / den : T(0);
                const T dkth = dnu * T(g.inv_pr);
                dk = {dnu, dnu, dkth, dkth};
            } else {
                dk = deardorff_diff(g, T(sqrt(s2a)), den > T(0) ? num / den : T(0), e);
            }
        }
    }
    const T trc = (cxx + czz) * T(1.0 / 3.0), trb = (bxx + bzz) * T(1.0 / 3.0);
    d[0] = T(2) * dk.mh * (cxx - trc) + T(2) * ka.mh * (bxx - trb);
    d[1] = T(2) * dk.mv * cxz + T(2) * ka.mv * bxz;
    d[2] = T(2) * dk.mv * (czz - trc) + T(2) * ka.mv * (bzz - trb);
    d[3] = dk.hh * txw + ka.hh * txb;
    d[4] = dk.hv * tzw + ka.hv * tzb;
}

// Jv at a point: out = 2v/dt - dF with dF from the pair (PW = u + e v, PB = v)
// and the derived differences.
template <int W, typename T, typename A, typename AD>
__device__ __forceinline__ void point_jv_pt(const Geo& g, const A& PW, const A& PB, const AD& D, int gz, T e, T ihx,
                                            T ihz, T o[4]) {
    const T* pbar = Bg<T>::pbar(g);
    const T* dpb = Bg<T>::dpbar(g);
    const T uB = PB.at(0, 0, 0), wB = PB.at(1, 0, 0), pB = PB.at(2, 0, 0), tB = PB.at(3, 0, 0);
    const T uA = PW.at(0, 0, 0) - e * uB, wA = PW.at(1, 0, 0) - e * wB, pA = PW.at(2, 0, 0) - e * pB;
    const T divW = acc_dx<W>(PW, 0, ihx) + acc_dz<W>(PW, 1, ihz);
    const T divB = acc_dx<W>(PB, 0, ihx) + acc_dz<W>(PB, 1, ihz);
    T cc[4] = {0, 0, 0, 0};
    if (g.convection) {
        // 1/2 [ D_j(a_j phi_b + b_j phi_w) + a_j D_j phi_b + b_j D_j phi_w ],  w = a + e b
        // (the tap values of a_j are the same for every field)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            auto px = [&](int q) {
                return (PW.at(0, 0, q) - e * PB.at(0, 0, q)) * PB.at(k, 0, q) + PB.at(0, 0, q) * PW.at(k, 0, q);
            };
            auto pz = [&](int q) {
                return (PW.at(1, q, 0) - e * PB.at(1, q, 0)) * PB.at(k, q, 0) + PB.at(1, q, 0) * PW.at(k, q, 0);
            };
            const T fx = dtaps<W>(px, ihx);
            const T fz = dtaps<W>(pz, ihz);
            const T dWx = acc_dx<W>(PW, k, ihx), dWz = acc_dz<W>(PW, k, ihz);
            const T dBx = acc_dx<W>(PB, k, ihx), dBz = acc_dz<W>(PB, k, ihz);
            const T ad = uA * dBx + wA * dBz + uB * dWx + wB * dWz;
            cc[k] = T(0.5) * (fx + fz + ad);
        }
    }
    const T th0 = T(g.theta0);
    const T dFu = -th0 * acc_dx<W>(PB, 2, ihx) + acc_dx<W>(D, 0, ihx) + acc_dz<W>(D, 1, ihz) - cc[0];
    const T dFw = -th0 * acc_dz<W>(PB, 2, ihz) + acc_dx<W>(D, 1, ihx) + acc_dz<W>(D, 2, ihz) - cc[1] +
                  T(g.g_theta0) * tB;
    T dFp;
    if (g.energy_test)
        dFp = -cc[2] - T(g.kappa_cp) * divB;
    else
        dFp = -cc[2] - wB * dpb[gz] - T(g.kappa) * ((pbar[gz] + pA) * divB + pB * divW);
    const T dFt = acc_dx<W>(D, 3, ihx) + acc_dz<W>(D, 4, ihz) - cc[3] - T(g.beta) * wB;
    const T tdt = T(g.two_dt);
    o[0] = tdt * uB - dFu;
    o[1] = tdt * wB - dFw;
    o[2] = tdt * pB - dFp;
    o[3] = tdt * tB - dFt;
}

// out = F (what 0), 2u/dt + F (1) or 2u/dt - F - f (2) at grid point (gz, gx)
template <typename T>
__device__ __forceinline__ void write_F(const Geo& g, const T* __restrict__ f, T* __restrict__ out, int gz, int gx,
                                        const T uv[4], const T Fv[4], int what) {
    const long long np = g.npts;
    const long long off = (long long)gz * g.nx + gx;
    T Fs[4] = {Fv[0], Fv[1], Fv[2], Fv[3]};
    if (gz == 0 && !g.energy_test) Fs[3] += Bg<T>::sflux(g)[gx];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T r;
        if (what == 0) r = Fs[k];
        else if (what == 1) r = T(g.two_dt) * uv[k] + Fs[k];
        else r = T(g.two_dt) * uv[k] - Fs[k] - (f ? f[k * np + off] : T(0));
        out[k * np + off] = r;
    }
}

// ---------------------------------------------------------------------------
// F(u) and the residual: one TX x TZ tile
// ---------------------------------------------------------------------------
template <typename T, int TX, int TZ, int W = 2>
__device__ __forceinline__ void apply_F_tile(const Geo& g, int x0, int z0, const T* __restrict__ u,
                                             const T* __restrict__ f, T* __restrict__ out, int what) {
    constexpr int H = 2 * W;
    constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H, PS = SZ * SX;
    constexpr int DX = TX + 2 * W, DZ = TZ + 2 * W, DS = DZ * DX;
    __shared__ T sp[4 * PS];
    __shared__ T sd[5 * DS];
    const T ihx = T(g.idx), ihz = T(g.idz);

    stage_fields<T, TX, TZ, 4, H>(g, u, sp, x0, z0, 0);
    __syncthreads();

    // stress and heat flux on the ring-W extended tile
    for (int idx = threadIdx.x; idx < DS; idx += blockDim.x) {
        const int z = idx / DX + W, x = idx - (idx / DX) * DX + W;
        const TileAcc<T, PS, SX> P{sp + z * SX + x};
        T d[5];
        derived_F_pt<W>(g, P, ihx, ihz, d);
#pragma unroll
        for (int k = 0; k < 5; ++k) sd[k * DS + idx] = d[k];
    }
    __syncthreads();

    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const TileAcc<T, PS, SX> P{sp + (lz + H) * SX + lx + H};
        const TileAcc<T, DS, DX> D{sd + (lz + W) * DX + lx + W};
        T Fv[4];
        point_F_pt<W>(g, P, D, gz, ihx, ihz, Fv);
        const T uv[4] = {P.at(0, 0, 0), P.at(1, 0, 0), P.at(2, 0, 0), P.at(3, 0, 0)};
        write_F(g, f, out, gz, gx, uv, Fv, what);
    }
}

// ---------------------------------------------------------------------------
// Jacobian-vector product: one TX x TZ tile
// ---------------------------------------------------------------------------
template <typename T, int TX, int TZ, int W = 2>
__device__ __forceinline__ void jv_tile(const Geo& g, int x0, int z0, const T* __restrict__ u,
                                        const T* __restrict__ v, double eps_in, const double* __restrict__ eps_dev,
                                        T* __restrict__ out) {
    constexpr int H = 2 * W;
    constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H;
    constexpr int DX = TX + 2 * W, DZ = TZ + 2 * W;
    constexpr int PS = SZ * SX, DS = DZ * DX;
    __shared__ T sa[4 * PS];   // u + e v
    __shared__ T sb[4 * PS];   // v
    __shared__ T sd[5 * DS];
    const T ihx = T(g.idx), ihz = T(g.idz);
    const T e = T(eps_dev ? *eps_dev : eps_in);

    {
        TileStage<T, TX, TZ, 4, H> st_a, st_b;
        st_a.load(g, u, x0, z0, 0);
        st_b.load(g, v, x0, z0, 0);
        st_a.store_sum(sa, st_b, e);
        st_b.store(sb);
    }
    __syncthreads();

    for (int idx = threadIdx.x; idx < DS; idx += blockDim.x) {
        const int z = idx / DX + W, x = idx - (idx / DX) * DX + W;
        const TileAcc<T, PS, SX> PA{sa + z * SX + x}, PB{sb + z * SX + x};
        T d[5];
        derived_jv_pt<W>(g, PA, PB, e, ihx, ihz, d);
#pragma unroll
        for (int k = 0; k < 5; ++k) sd[k * DS + idx] = d[k];
    }
    __syncthreads();

    const long long np = g.npts;
    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const int c = (lz + H) * SX + lx + H;
        const TileAcc<T, PS, SX> PA{sa + c}, PB{sb + c};
        const TileAcc<T, DS, DX> D{sd + (lz + W) * DX + lx + W};
        T o[4];
        point_jv_pt<W>(g, PA, PB, D, gz, e, ihx, ihz, o);
        const long long off = (long long)gz * g.nx + gx;
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k * np + off] = o[k];
    }
}

// ---------------------------------------------------------------------------
// Physics-based preconditioner
// ---------------------------------------------------------------------------
// Frozen eddy viscosity on the grid extended by a ring of W, stored with row
// stride nx + 2W: ghost values are formed from the mirrored velocity, like every
// derived quantity (at a no-slip bottom they are not a mirror image of the
// interior values).
template <typename T, int W = 2>
__device__ __forceinline__ void frozen_nu_point(const Geo& g, long long i, const T* __restrict__ u,
                                                T* __restrict__ nu) {
    const int ex = g.nx + 2 * W, ez = g.nz + 2 * W;
    if (i >= (long long)ex * ez) return;
    const int gx = (int)(i % ex) - W, gz = (int)(i / ex) - W;
    const long long np = g.npts;
    auto val = [&](int f, int x, int z) {
        int sx, sz;
        const int mx = map_axis(x, g.nx, g.bcl == JFNK_BC_PERIODIC, sx);
        const int mz = map_axis(z, g.nz, g.bcv == JFNK_BC_PERIODIC, sz);
        const T v = u[(long long)f * np + (long long)mz * g.nx + mx];
        return sign2d(f, sx, sz, g.bcv) < 0 ? -v : v;
    };
    const T ihx = T(g.idx), ihz = T(g.idz);
    const T ux = dtaps<W>([&](int o) { return val(0, gx + o, gz); }, ihx);
    const T uz = dtaps<W>([&](int o) { return val(0, gx, gz + o); }, ihz);
    const T wx = dtaps<W>([&](int o) { return val(1, gx + o, gz); }, ihx);
    const T wz = dtaps<W>([&](int o) { return val(1, gx, gz + o); }, ihz);
    const T sxz = T(0.5) * (uz + wx);
    const T s2 = ux * ux + wz * wz + T(2) * sxz * sxz;
    T n, k;
    closure_coeffs(g, s2, n, k);
    nu[i] = n;
}

// Frozen coefficients of the preconditioner from the frozen viscosity nu_pt
// (for the anisotropic closure the Smagorinsky nu, |S| = nu dd_inv_nu).
template <typename T>
__device__ __forceinline__ Coef<T> pc_coef(const Geo& g, T nu_pt) {
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
        const T kth = nu_pt * T(g.inv_pr);
        return {nu_pt, nu_pt, kth, kth};
    }
    if (g.closure == JFNK_CLOSURE_CONST_K) return {T(g.k_m), T(g.k_m), T(g.k_h), T(g.k_h)};
    if (g.closure == JFNK_CLOSURE_DEARDORFF) return deardorff_coef(g, nu_pt * T(g.dd_inv_nu));
    return {T(0), T(0), T(0), T(0)};
}

// Diagonal of a field block: 2/dt + 2 sum_m c_m^2 (K_h/dx^2 + K_v/dz^2) (65/72 for
// the 5-point stencil); one K times (1/dx^2 + 1/dz^2) for isotropic closures.
template <typename T, int W>
__device__ __forceinline__ T pc_block_diag(const Geo& g, T kh, T kv) {
    const T cD = T(DW<W>::sumsq2);
    if (g.closure == JFNK_CLOSURE_DEARDORFF) return T(g.two_dt) + cD * (kh * T(g.idx * g.idx) + kv * T(g.idz * g.idz));
    return T(g.two_dt) + cD * kh * T(g.idx * g.idx + g.idz * g.idz);
}

// Start of the Jacobi iteration, z0 = v / d, fused with the normalisation of
// the incoming Krylov vector (v = V_j / *div written back) and, when no sweep
// follows, the norm of z for the finite-difference step.
// Returns this thread's contribution to ||z||^2.
template <typename T, int W = 2>
__device__ __forceinline__ double pc_diag_point(const Geo& g, long long i, const T* __restrict__ nu,
                                                T* __restrict__ vj, const double* __restrict__ div,
                                                T* __restrict__ z) {
    double acc = 0.0;
    if (i < g.npts) {
        const long long ie = (i / g.nx + W) * (long long)(g.nx + 2 * W) + (i % g.nx) + W;
        const Coef<T> k = pc_coef(g, nu[ie]);
        const T dm = pc_block_diag<T, W>(g, k.mh, k.mv);
        const T dd[4] = {dm, dm, T(g.two_dt), pc_block_diag<T, W>(g, k.hh, k.hv)};
        const long long np = g.npts;
        const double dv = div ? *div : 1.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T v = vj[k * np + i];
            if (div) {
                v = (T)((double)v / dv);
                vj[k * np + i] = v;
            }
            const T zz = v / dd[k];
            z[k * np + i] = zz;
            acc += (double)zz * (double)zz;
        }
    }
    return acc;
}

// Returns this thread's contribution to ||zout||^2.
template <typename T, int TX, int TZ, int W = 2>
__device__ __forceinline__ double pc_sweep_tile(const Geo& g, int x0, int z0, const T* __restrict__ u,
                                                const T* __restrict__ nu, const T* __restrict__ r,
                                                const T* __restrict__ zin, T* __restrict__ zout) {
    constexpr int H = 2 * W;
    constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H, PS = SZ * SX;
    constexpr int DX = TX + 2 * W, DZ = TZ + 2 * W, DS = DZ * DX;
    __shared__ T sz_[4 * PS];   // z, halo 2W
    __shared__ T sv[2 * DS];    // frozen velocity, halo W
    __shared__ T sn[DS];        // frozen viscosity, halo W
    __shared__ T sf[6 * DS];    // K D_x z, K D_z z for u, w, theta on ring W
    double zacc = 0.0;
    const T ihx = T(g.idx), ihz = T(g.idz);
    const long long np = g.npts;

    {
        // every global load of the tile issued before the LDS stores
        TileStage<T, TX, TZ, 4, H> st;
        st.load(g, zin, x0, z0, 0);
        constexpr int DIT = (DS + kTileThreads - 1) / kTileThreads;
        T a0[DIT], a1[DIT], nn[DIT];
        unsigned sgn = 0u;
#pragma unroll
        for (int it = 0; it < DIT; ++it) {
            const int idx = min((int)threadIdx.x + it * kTileThreads, DS - 1);
            const int lz = idx / DX, lx = idx - lz * DX;
            int sx, szd;
            const int gx = map_axis(x0 + lx - W, g.nx, g.bcl == JFNK_BC_PERIODIC, sx);
            const int gz = map_axis(z0 + lz - W, g.nz, g.bcv == JFNK_BC_PERIODIC, szd);
            const long long off = (long long)gz * g.nx + gx;
            a0[it] = u[off];
            a1[it] = u[np + off];
            if (sign2d(0, sx, szd, g.bcv) < 0) sgn |= 1u << (2 * it);
            if (sign2d(1, sx, szd, g.bcv) < 0) sgn |= 1u << (2 * it + 1);
            // extended viscosity: row gz + W of the (nz + 2W) x (nx + 2W) ring-W grid
            const int ex = min(max(x0 + lx, 0), g.nx + 2 * W - 1), ez = min(max(z0 + lz, 0), g.nz + 2 * W - 1);
            nn[it] = nu[(long long)ez * (g.nx + 2 * W) + ex];
        }
        st.store(sz_);
#pragma unroll
        for (int it = 0; it < DIT; ++it) {
            const int idx = (int)threadIdx.x + it * kTileThreads;
            if (idx < DS) {
                sv[idx] = (sgn >> (2 * it)) & 1u ? -a0[it] : a0[it];
                sv[DS + idx] = (sgn >> (2 * it + 1)) & 1u ? -a1[it] : a1[it];
                sn[idx] = nn[it];
            }
        }
    }
    __syncthreads();

    for (int idx = threadIdx.x; idx < DS; idx += blockDim.x) {
        const int z = idx / DX + W, x = idx - (idx / DX) * DX + W;
        const Coef<T> k = pc_coef(g, sn[idx]);
        const T* zu = sz_;
        const T* zw = sz_ + PS;
        const T* zt = sz_ + 3 * PS;
        sf[0 * DS + idx] = k.mh * dx_s<T, SX, W>(zu, z, x, ihx);
        sf[1 * DS + idx] = k.mv * dz_s<T, SX, W>(zu, z, x, ihz);
        sf[2 * DS + idx] = k.mh * dx_s<T, SX, W>(zw, z, x, ihx);
        sf[3 * DS + idx] = k.mv * dz_s<T, SX, W>(zw, z, x, ihz);
        sf[4 * DS + idx] = k.hh * dx_s<T, SX, W>(zt, z, x, ihx);
        sf[5 * DS + idx] = k.hv * dz_s<T, SX, W>(zt, z, x, ihz);
    }
    __syncthreads();

    const bool conv = g.convection != 0;
    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const int z = lz + H, x = lx + H;
        const int dzi = lz + W, dxi = lx + W;
        const int dc = dzi * DX + dxi;
        const T a = sv[dc], w = sv[DS + dc];
        const Coef<T> kc = pc_coef(g, sn[dc]);
        const T dmom = pc_block_diag<T, W>(g, kc.mh, kc.mv), dth = pc_block_diag<T, W>(g, kc.hh, kc.hv);
        const long long off = (long long)gz * g.nx + gx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T* Z = sz_ + k * PS;
            const T zc = Z[z * SX + x];
            T diff = T(0);
            if (k != 2) {
                const int fi = (k == 3) ? 4 : 2 * k;
                diff = dx_s<T, DX, W>(sf + fi * DS, dzi, dxi, ihx) + dz_s<T, DX, W>(sf + (fi + 1) * DS, dzi, dxi, ihz);
            }
            T cv = T(0);
            if (conv) {
                const T* va = sv;
                const T* vw = sv + DS;
                // D_x(a z): products over the ring-2 velocity and halo-4 z
                auto pxv = [&](int o) { return va[dc + o] * Z[z * SX + x + o]; };
                auto pzv = [&](int o) { return vw[dc + o * DX] * Z[(z + o) * SX + x]; };
                const T fx = dtaps<W>(pxv, ihx);
                const T fz = dtaps<W>(pzv, ihz);
                cv = T(0.5) * (fx + fz + a * dx_s<T, SX, W>(Z, z, x, ihx) + w * dz_s<T, SX, W>(Z, z, x, ihz));
            }
            const T Pz = T(g.two_dt) * zc + (cv - diff);
            const T d = k == 2 ? T(g.two_dt) : (k == 3 ? dth : dmom);
            const T zn = zc + (r[k * np + off] - Pz) / d;
            zout[k * np + off] = zn;
            zacc += (double)zn * (double)zn;
        }
    }
    return zacc;
}

}  // namespace s2d
}  // namespace jfnk
