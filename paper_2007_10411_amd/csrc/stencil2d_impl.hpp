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

namespace jfnk {
namespace s2d {


constexpr int kHalo = 4;

// Source index of extended position e along an axis of n points, and which
// ghost side it came from (0 interior, 1 low, 2 high).  Positions further out
// than the halo are clamped (they only feed outputs outside the domain).
__device__ __forceinline__ int map_axis(int e, int n, bool periodic, int& side) {
    side = 0;
    if (periodic) {
        int r = e % n;
        return r < 0 ? r + n : r;
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
    return (T(2.0 / 3.0) * (p1 - m1) - T(1.0 / 12.0) * (p2 - m2)) * ih;
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
        for (int m = 0; m < W; ++m) acc += T(DW<W>::c[m]) * (f(m + 1) - f(-m - 1));
        return acc * ih;
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
};

// Stage the n-field state (field stride np) with halo H into LDS s[f][SZ][SX].
template <typename T, int TX, int TZ, int NFL, int H = kHalo>
__device__ __forceinline__ void stage_fields(const Geo& g, const T* __restrict__ u, T* s, int x0, int z0,
                                             int f_first) {
    TileStage<T, TX, TZ, NFL, H> st;
    st.load(g, u, x0, z0, f_first);
    st.store(s);
}

template <typename T>
__device__ __forceinline__ void closure_coeffs(const Geo& g, T s2, T& nu, T& kth) {
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
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

// ---------------------------------------------------------------------------
// F(u) and the residual
// ---------------------------------------------------------------------------
template <typename T, int TX, int TZ, int W = 2>
__device__ __forceinline__ void apply_F_tile(const Geo& g, int x0, int z0, const T* __restrict__ u,
                                             const T* __restrict__ f, T* __restrict__ out, int what) {
    constexpr int H = 2 * W;
    constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H;
    constexpr int DX = TX + 2 * W, DZ = TZ + 2 * W;
    __shared__ T sp[4 * SZ * SX];
    __shared__ T sd[5 * DZ * DX];
    const T ihx = T(g.idx), ihz = T(g.idz);

    stage_fields<T, TX, TZ, 4, H>(g, u, sp, x0, z0, 0);
    __syncthreads();

    const T* su = sp;
    const T* sw = sp + SZ * SX;
    const T* spp = sp + 2 * SZ * SX;
    const T* sth = sp + 3 * SZ * SX;

    // stress and heat flux on the ring-W extended tile
    for (int idx = threadIdx.x; idx < DZ * DX; idx += blockDim.x) {
        const int dzi = idx / DX, dxi = idx - (idx / DX) * DX;
        const int z = dzi + W, x = dxi + W;
        const T ux = dx_s<T, SX, W>(su, z, x, ihx), uz = dz_s<T, SX, W>(su, z, x, ihz);
        const T wx = dx_s<T, SX, W>(sw, z, x, ihx), wz = dz_s<T, SX, W>(sw, z, x, ihz);
        const T tx = dx_s<T, SX, W>(sth, z, x, ihx), tz = dz_s<T, SX, W>(sth, z, x, ihz);
        const T sxz = T(0.5) * (uz + wx);
        const T div = ux + wz;
        const T s2 = ux * ux + wz * wz + T(2) * sxz * sxz;
        T nu, kth;
        closure_coeffs(g, s2, nu, kth);
        const T third = div / T(3);
        sd[0 * DZ * DX + idx] = T(2) * nu * (ux - third);
        sd[1 * DZ * DX + idx] = T(2) * nu * sxz;
        sd[2 * DZ * DX + idx] = T(2) * nu * (wz - third);
        sd[3 * DZ * DX + idx] = kth * tx;
        sd[4 * DZ * DX + idx] = kth * tz;
    }
    __syncthreads();

    const long long np = g.npts;
    const T* pb = Bg<T>::pbar(g);
    const T* dpb = Bg<T>::dpbar(g);
    const T* sfl = Bg<T>::sflux(g);
    const bool conv = g.convection != 0;
    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const int z = lz + H, x = lx + H;              // primitive coordinates
        const int dz_ = lz + W, dx_ = lx + W;          // derived coordinates
        const T uu = su[z * SX + x], ww = sw[z * SX + x], pp = spp[z * SX + x], th = sth[z * SX + x];
        const T ux = dx_s<T, SX, W>(su, z, x, ihx), wz = dz_s<T, SX, W>(sw, z, x, ihz);
        const T div = ux + wz;
        T cu = 0, cw = 0, cp = 0, ct = 0;
        if (conv) {
            const T uz = dz_s<T, SX, W>(su, z, x, ihz), wx = dx_s<T, SX, W>(sw, z, x, ihx);
            const T px = dx_s<T, SX, W>(spp, z, x, ihx), pz = dz_s<T, SX, W>(spp, z, x, ihz);
            const T tx = dx_s<T, SX, W>(sth, z, x, ihx), tz = dz_s<T, SX, W>(sth, z, x, ihz);
            cu = T(0.5) * (dx_prod<T, SX, W>(su, su, z, x, ihx) + dz_prod<T, SX, W>(sw, su, z, x, ihz) + uu * ux + ww * uz);
            cw = T(0.5) * (dx_prod<T, SX, W>(su, sw, z, x, ihx) + dz_prod<T, SX, W>(sw, sw, z, x, ihz) + uu * wx + ww * wz);
            cp = T(0.5) * (dx_prod<T, SX, W>(su, spp, z, x, ihx) + dz_prod<T, SX, W>(sw, spp, z, x, ihz) + uu * px + ww * pz);
            ct = T(0.5) * (dx_prod<T, SX, W>(su, sth, z, x, ihx) + dz_prod<T, SX, W>(sw, sth, z, x, ihz) + uu * tx + ww * tz);
        }
        const T* txx = sd;
        const T* txz = sd + DZ * DX;
        const T* tzz = sd + 2 * DZ * DX;
        const T* qx = sd + 3 * DZ * DX;
        const T* qz = sd + 4 * DZ * DX;
        const T th0 = T(g.theta0);
        T Fu = -th0 * dx_s<T, SX, W>(spp, z, x, ihx) + dx_s<T, DX, W>(txx, dz_, dx_, ihx) + dz_s<T, DX, W>(txz, dz_, dx_, ihz) - cu;
        T Fw = -th0 * dz_s<T, SX, W>(spp, z, x, ihz) + dx_s<T, DX, W>(txz, dz_, dx_, ihx) + dz_s<T, DX, W>(tzz, dz_, dx_, ihz) - cw +
               T(g.g_theta0) * th;
        T Fp;
        if (g.energy_test)
            Fp = -cp - T(g.kappa_cp) * div;
        else
            Fp = -cp - ww * dpb[gz] - T(g.kappa) * (pb[gz] + pp) * div;
        T Ft = dx_s<T, DX, W>(qx, dz_, dx_, ihx) + dz_s<T, DX, W>(qz, dz_, dx_, ihz) - ct - T(g.beta) * ww;
        if (gz == 0 && !g.energy_test) Ft += sfl[gx];
        const long long off = (long long)gz * g.nx + gx;
        T Fv[4] = {Fu, Fw, Fp, Ft};
        const T uv[4] = {uu, ww, pp, th};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T r;
            if (what == 0) r = Fv[k];
            else if (what == 1) r = T(g.two_dt) * uv[k] + Fv[k];
            else r = T(g.two_dt) * uv[k] - Fv[k] - (f ? f[k * np + off] : T(0));
            out[k * np + off] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// Jacobian-vector product, stable finite-difference form
//   [B(a + e b, c + e d) - B(a, c)] / e = B(a, d) + B(b, c) + e B(b, d)
//   nu difference: (cs Delta)^2 sqrt2 (2 S:T + e T:T) / (|S + e T| + |S|)
// ---------------------------------------------------------------------------
template <typename T, int TX, int TZ, int W = 2>
__device__ __forceinline__ void jv_tile(const Geo& g, int x0, int z0, const T* __restrict__ u,
                                        const T* __restrict__ v, double eps_in, const double* __restrict__ eps_dev,
                                        T* __restrict__ out) {
    constexpr int H = 2 * W;
    constexpr int SX = TX + 2 * H, SZ = TZ + 2 * H;
    constexpr int DX = TX + 2 * W, DZ = TZ + 2 * W;
    constexpr int PS = SZ * SX, DS = DZ * DX;
    __shared__ T sa[4 * PS];
    __shared__ T sb[4 * PS];
    __shared__ T sd[5 * DS];
    const T ihx = T(g.idx), ihz = T(g.idz);
    const T e = T(eps_dev ? *eps_dev : eps_in);

    {
        TileStage<T, TX, TZ, 4, H> st_a, st_b;
        st_a.load(g, u, x0, z0, 0);
        st_b.load(g, v, x0, z0, 0);
        st_a.store(sa);
        st_b.store(sb);
    }
    __syncthreads();

    const T *ua = sa, *wa = sa + PS, *pa = sa + 2 * PS, *ta = sa + 3 * PS;
    const T *ub = sb, *wb = sb + PS, *pbv = sb + 2 * PS, *tb = sb + 3 * PS;

    for (int idx = threadIdx.x; idx < DS; idx += blockDim.x) {
        const int z = idx / DX + W, x = idx - (idx / DX) * DX + W;
        const T uxa = dx_s<T, SX, W>(ua, z, x, ihx), uza = dz_s<T, SX, W>(ua, z, x, ihz);
        const T wxa = dx_s<T, SX, W>(wa, z, x, ihx), wza = dz_s<T, SX, W>(wa, z, x, ihz);
        const T uxb = dx_s<T, SX, W>(ub, z, x, ihx), uzb = dz_s<T, SX, W>(ub, z, x, ihz);
        const T wxb = dx_s<T, SX, W>(wb, z, x, ihx), wzb = dz_s<T, SX, W>(wb, z, x, ihz);
        const T txa = dx_s<T, SX, W>(ta, z, x, ihx), tza = dz_s<T, SX, W>(ta, z, x, ihz);
        const T txb = dx_s<T, SX, W>(tb, z, x, ihx), tzb = dz_s<T, SX, W>(tb, z, x, ihz);
        // strain of u (a) and of v (b)
        const T axx = uxa, azz = wza, axz = T(0.5) * (uza + wxa);
        const T bxx = uxb, bzz = wzb, bxz = T(0.5) * (uzb + wxb);
        T nua, ktha, dnu, dkth;
        const T s2a = axx * axx + azz * azz + T(2) * axz * axz;
        closure_coeffs(g, s2a, nua, ktha);
        // strain of u + e v
        const T cxx = axx + e * bxx, czz = azz + e * bzz, cxz = axz + e * bxz;
        if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
            const T sab = axx * bxx + azz * bzz + T(2) * axz * bxz;
            const T sbb = bxx * bxx + bzz * bzz + T(2) * bxz * bxz;
            const T s2c = cxx * cxx + czz * czz + T(2) * cxz * cxz;
            const T den = sqrt(s2a) + sqrt(s2c);
            const T num = T(2) * sab + e * sbb;
            dnu = den > T(0) ? T(g.smag) * T(1.4142135623730951) * num / den : T(0);
            dkth = dnu * T(g.inv_pr);
        } else {
            dnu = T(0);
            dkth = T(0);
        }
        const T trc = (cxx + czz) / T(3), trb = (bxx + bzz) / T(3);
        sd[0 * DS + idx] = T(2) * dnu * (cxx - trc) + T(2) * nua * (bxx - trb);
        sd[1 * DS + idx] = T(2) * dnu * cxz + T(2) * nua * bxz;
        sd[2 * DS + idx] = T(2) * dnu * (czz - trc) + T(2) * nua * (bzz - trb);
        sd[3 * DS + idx] = dkth * (txa + e * txb) + ktha * txb;
        sd[4 * DS + idx] = dkth * (tza + e * tzb) + ktha * tzb;
    }
    __syncthreads();

    const long long np = g.npts;
    const T* pbar = Bg<T>::pbar(g);
    const T* dpb = Bg<T>::dpbar(g);
    const bool conv = g.convection != 0;
    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const int z = lz + H, x = lx + H;
        const int dz_ = lz + W, dx_ = lx + W;
        const int c = z * SX + x;
        const T uA = ua[c], wA = wa[c], pA = pa[c];
        const T uB = ub[c], wB = wb[c], pB = pbv[c], tB = tb[c];
        const T divA = dx_s<T, SX, W>(ua, z, x, ihx) + dz_s<T, SX, W>(wa, z, x, ihz);
        const T divB = dx_s<T, SX, W>(ub, z, x, ihx) + dz_s<T, SX, W>(wb, z, x, ihz);
        T cu = 0, cw = 0, cp = 0, ct = 0;
        if (conv) {
            // 1/2 [ D_j(a_j phi_b + b_j phi_a + e b_j phi_b) + a_j D_j phi_b + b_j D_j phi_a + e b_j D_j phi_b ]
            const T* fa[4] = {ua, wa, pa, ta};
            const T* fb[4] = {ub, wb, pbv, tb};
            T cc[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T* A = fa[k];
                const T* B = fb[k];
                auto px = [&](int o) { return ua[c + o] * B[c + o] + ub[c + o] * (A[c + o] + e * B[c + o]); };
                auto pz = [&](int o) { return wa[c + o] * B[c + o] + wb[c + o] * (A[c + o] + e * B[c + o]); };
                const T fx = dtaps<W>(px, ihx);
                const T fz = dtaps<W>([&](int o) { return pz(o * SX); }, ihz);
                const T dAx = dx_s<T, SX, W>(A, z, x, ihx), dAz = dz_s<T, SX, W>(A, z, x, ihz);
                const T dBx = dx_s<T, SX, W>(B, z, x, ihx), dBz = dz_s<T, SX, W>(B, z, x, ihz);
                const T ad = uA * dBx + wA * dBz + uB * (dAx + e * dBx) + wB * (dAz + e * dBz);
                cc[k] = T(0.5) * (fx + fz + ad);
            }
            cu = cc[0];
            cw = cc[1];
            cp = cc[2];
            ct = cc[3];
        }
        const T *txx = sd, *txz = sd + DS, *tzz = sd + 2 * DS, *qx = sd + 3 * DS, *qz = sd + 4 * DS;
        const T th0 = T(g.theta0);
        const T dFu = -th0 * dx_s<T, SX, W>(pbv, z, x, ihx) + dx_s<T, DX, W>(txx, dz_, dx_, ihx) +
                      dz_s<T, DX, W>(txz, dz_, dx_, ihz) - cu;
        const T dFw = -th0 * dz_s<T, SX, W>(pbv, z, x, ihz) + dx_s<T, DX, W>(txz, dz_, dx_, ihx) +
                      dz_s<T, DX, W>(tzz, dz_, dx_, ihz) - cw + T(g.g_theta0) * tB;
        T dFp;
        if (g.energy_test)
            dFp = -cp - T(g.kappa_cp) * divB;
        else
            dFp = -cp - wB * dpb[gz] - T(g.kappa) * ((pbar[gz] + pA) * divB + pB * divA + e * pB * divB);
        const T dFt = dx_s<T, DX, W>(qx, dz_, dx_, ihx) + dz_s<T, DX, W>(qz, dz_, dx_, ihz) - ct - T(g.beta) * wB;
        const long long off = (long long)gz * g.nx + gx;
        const T tdt = T(g.two_dt);
        out[off] = tdt * uB - dFu;
        out[np + off] = tdt * wB - dFw;
        out[2 * np + off] = tdt * pB - dFp;
        out[3 * np + off] = tdt * tB - dFt;
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

// Diagonal of the field block: 2/dt + 2 sum_m c_m^2 K (1/dx^2 + 1/dz^2) (65/72
// for the 5-point stencil).
template <typename T>
__device__ __forceinline__ void pc_coeffs(const Geo& g, T nu_pt, T& kmom, T& kth) {
    if (g.closure == JFNK_CLOSURE_SMAGORINSKY) {
        kmom = nu_pt;
        kth = nu_pt * T(g.inv_pr);
    } else if (g.closure == JFNK_CLOSURE_CONST_K) {
        kmom = T(g.k_m);
        kth = T(g.k_h);
    } else {
        kmom = T(0);
        kth = T(0);
    }
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
        T km, kt;
        pc_coeffs(g, nu[ie], km, kt);
        const T ih2 = T(g.idx * g.idx + g.idz * g.idz);
        const T cD = T(DW<W>::sumsq2);
        const T dd[4] = {T(g.two_dt) + cD * km * ih2, T(g.two_dt) + cD * km * ih2, T(g.two_dt),
                         T(g.two_dt) + cD * kt * ih2};
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
        T km, kt;
        pc_coeffs(g, sn[idx], km, kt);
        const T* zu = sz_;
        const T* zw = sz_ + PS;
        const T* zt = sz_ + 3 * PS;
        sf[0 * DS + idx] = km * dx_s<T, SX, W>(zu, z, x, ihx);
        sf[1 * DS + idx] = km * dz_s<T, SX, W>(zu, z, x, ihz);
        sf[2 * DS + idx] = km * dx_s<T, SX, W>(zw, z, x, ihx);
        sf[3 * DS + idx] = km * dz_s<T, SX, W>(zw, z, x, ihz);
        sf[4 * DS + idx] = kt * dx_s<T, SX, W>(zt, z, x, ihx);
        sf[5 * DS + idx] = kt * dz_s<T, SX, W>(zt, z, x, ihz);
    }
    __syncthreads();

    const bool conv = g.convection != 0;
    const T ih2 = T(g.idx * g.idx + g.idz * g.idz);
    const T cD = T(DW<W>::sumsq2);
    for (int idx = threadIdx.x; idx < TZ * TX; idx += blockDim.x) {
        const int lz = idx / TX, lx = idx - (idx / TX) * TX;
        const int gx = x0 + lx, gz = z0 + lz;
        if (gx >= g.nx || gz >= g.nz) continue;
        const int z = lz + H, x = lx + H;
        const int dzi = lz + W, dxi = lx + W;
        const int dc = dzi * DX + dxi;
        const T a = sv[dc], w = sv[DS + dc];
        T km, kt;
        pc_coeffs(g, sn[dc], km, kt);
        const long long off = (long long)gz * g.nx + gx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T* Z = sz_ + k * PS;
            const T zc = Z[z * SX + x];
            T diff = T(0);
            T kk = (k == 2) ? T(0) : (k == 3 ? kt : km);
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
            const T d = T(g.two_dt) + cD * kk * ih2;
            const T zn = zc + (r[k * np + off] - Pz) / d;
            zout[k * np + off] = zn;
            zacc += (double)zn * (double)zn;
        }
    }
    return zacc;
}

}  // namespace s2d
}  // namespace jfnk
