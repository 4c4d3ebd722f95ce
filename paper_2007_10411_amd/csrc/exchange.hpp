// Anisotropic exchange coefficients (section 2.4, Eq. 7) shared by the 2D and
// 3D stencil kernels.  With eps^(1/3) = (cs Delta)^(2/3) 2^(1/6) |S| every
// coefficient is linear in |S| = sqrt(S:S) below the mixing-length cap:
//   K_m = dd_ah |S|, K_M = dd_av |S|, l = min(dd_b |S|, dd_delta),
//   K_h = K_m + dd_ch l |S|, K_H = K_M + dd_cv l |S|
// (constants set on the host; dd_b = 0 at N = 0, where l = dd_delta).

#pragma once

#include "jfnk_internal.hpp"

namespace jfnk {

// Momentum and heat exchange coefficients, horizontal and vertical.
template <typename T> struct Coef {
    T mh, mv, hh, hv;
};

// The constants in the arithmetic of T (FP32: the host-rounded copies, the
// same values as a conversion on the device).
template <typename T> struct DdK;
template <> struct DdK<double> {
    const Geo& g;
    __device__ __forceinline__ double ah() const { return g.dd_ah; }
    __device__ __forceinline__ double av() const { return g.dd_av; }
    __device__ __forceinline__ double ch() const { return g.dd_ch; }
    __device__ __forceinline__ double cv() const { return g.dd_cv; }
    __device__ __forceinline__ double b() const { return g.dd_b; }
    __device__ __forceinline__ double delta() const { return g.dd_delta; }
};
template <> struct DdK<float> {
    const Geo& g;
    __device__ __forceinline__ float ah() const { return g.f.dd_ah; }
    __device__ __forceinline__ float av() const { return g.f.dd_av; }
    __device__ __forceinline__ float ch() const { return g.f.dd_ch; }
    __device__ __forceinline__ float cv() const { return g.f.dd_cv; }
    __device__ __forceinline__ float b() const { return g.f.dd_b; }
    __device__ __forceinline__ float delta() const { return g.f.dd_delta; }
};

// Eq. 7 coefficients from |S| = sqrt(S:S): each is linear in |S| below the
// mixing-length cap (the constants are set on the host).
template <typename T>
__device__ __forceinline__ Coef<T> deardorff_coef(const Geo& g, T mag) {
    const DdK<T> k{g};
    const T l = g.dd_b > 0 ? min(k.b() * mag, k.delta()) : k.delta();
    const T km = k.ah() * mag, kM = k.av() * mag;
    return {km, kM, km + k.ch() * l * mag, kM + k.cv() * l * mag};
}

// [K(S + e T) - K(S)] / e of the Eq. 7 coefficients at |S| = magA, with
// dmag = (|S + e T| - |S|) / e formed stably; the mixing-length difference
// takes the side of the cap that S is on (no two nearly equal values are
// subtracted).  e = 0 gives the derivative.
template <typename T>
__device__ __forceinline__ Coef<T> deardorff_diff(const Geo& g, T magA, T dmag, T e) {
    const DdK<T> k{g};
    const T delta = k.delta();
    T lA = delta, dl = T(0);
    if (g.dd_b > 0) {
        const T b = k.b(), xA = b * magA;
        lA = min(xA, delta);
        if (e == T(0))
            dl = xA < delta ? b * dmag : (xA > delta ? T(0) : min(b * dmag, T(0)));
        else
            dl = xA >= delta ? min((xA - delta) / e + b * dmag, T(0)) : min(b * dmag, (delta - xA) / e);
    }
    const T lW = lA + e * dl;
    const T dlS = lW * dmag + magA * dl;   // (l_W |S_W| - l_A |S_A|) / e
    const T dkm = k.ah() * dmag, dkM = k.av() * dmag;
    return {dkm, dkM, dkm + k.ch() * dlS, dkM + k.cv() * dlS};
}

}  // namespace jfnk
