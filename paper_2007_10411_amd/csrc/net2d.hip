// Learned right preconditioner for the Krylov solve (2D): a 4-layer 3x3
// convolutional network applied as
//     z = (dt/2) r + s N(r / s),     s = RMS of r over all fields (1 if r = 0),
//     N = conv(nf->16) GELU conv(16->16) GELU conv(16->16) GELU conv(16->nf),
// 3x3 kernels with a dilation d_l per layer (taps at d_l * (-1, 0, 1), d_l <= 8),
// zero padding, erf GELU.  Inference runs in BF16 on MFMA
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation, one 3x3 tap per instruction,
// erf by a rational approximation inside the BF16 rounding); training
// (forward, backward, Adam on FP32 master weights) runs in FP32 with the
// exact erf.
//
// The FP32 training activations are channel-major [c][nz][nx] like the state
// vectors; the BF16 inference activations are pixel-major [pixel][16], so one
// pixel's channels are one 32-byte row.  Parameters
// are one flat FP32 vector: per layer W[co][ci][kz][kx] (tap offsets kz-1, kx-1)
// followed by b[co].

#include "jfnk_internal.hpp"
#include "reduce.hpp"
#include "stencil2d_impl.hpp"

#include <algorithm>
#include <cmath>

namespace jfnk {

namespace {

constexpr int kHid = 16;
constexpr int kTX = 64, kTZ = 4;            // output tile per 256-thread block
constexpr int kMaxDil = 8;
// the first layer finishes the input scale itself when k_field_sumsq leaves at
// most this many partial sums (a few per thread), saving a launch on small grids
constexpr int kFuseScalePartials = 1024;
constexpr int kSX = kTX + 2 * kMaxDil, kSZ = kTZ + 2 * kMaxDil;   // input tile with the largest halo

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {   // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
// GELU of the BF16 inference path: erf by the rational approximation 7.1.26 of
// Abramowitz and Stegun (absolute error below 1.5e-7), written through erfc,
// 1 + erf(x / sqrt2) = 2 - c or c with c = erfc(|x| / sqrt2), so that the
// negative tail keeps a relative error below 2e-3, inside the BF16 rounding
// (2^-8) of the activations.
__device__ __forceinline__ float gelu_fast(float x) {
    const float t = fabsf(x) * 0.70710678118654752f;
    const float k = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * t);
    const float poly =
        k * (0.254829592f + k * (-0.284496736f + k * (1.421413741f + k * (-1.453152027f + k * 1.061405429f))));
    const float c = poly * __expf(-t * t);
    return 0.5f * x * (x >= 0.0f ? 2.0f - c : c);
}
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
}

enum { L_FIRST = 0, L_MID = 1, L_LAST = 2 };

// ---------------------------------------------------------------------------
// scale s = sqrt(mean r^2) over all fields (stored once per field channel)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_field_sumsq(const float* __restrict__ r, long long npts,
                                                     double* __restrict__ partials) {
    __shared__ double red[4];
    const int f = blockIdx.y;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < npts; i += (long long)gridDim.x * 256) {
        const double v = r[f * npts + i];
        acc += v * v;
    }
    const double t = block_sum256(acc, red);
    if (threadIdx.x == 0) partials[(long long)f * gridDim.x + blockIdx.x] = t;
}

// partials: nsets sets of nblk per-block sums of squares (one set per field
// from k_field_sumsq, or one set over all fields); s[0..nf) = sqrt(sum / count)
__global__ __launch_bounds__(256) void k_field_scale(const double* __restrict__ partials, int nblk, int nsets,
                                                     double count, int nf, float* __restrict__ s) {
    __shared__ double red[4];
    double tot = 0.0;
    for (int f = 0; f < nsets; ++f) tot += sum_partials(partials + (long long)f * nblk, nblk, 1, 0, red);
    if (threadIdx.x == 0) {
        const double v = sqrt(tot / count);
        for (int f = 0; f < nf; ++f) s[f] = v > 0.0 ? (float)v : 1.0f;
    }
}

// ---------------------------------------------------------------------------
// FP32 convolution (training forward, backward-data via transposed weights)
// out_pre[co] = b[co] + sum_ci sum_taps W[co][ci][t] in[ci](p + off_t)
// FIRST: in = r / s;  MID: in = act;  LAST: z = (dt/2) r + s (out_pre)
// post = GELU(out_pre) for FIRST/MID (or, with gmul, out_pre * gelu'(gmul))
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_conv_f32(int nx, int nz, const float* __restrict__ in, int cin,
                                                  const float* __restrict__ W, const float* __restrict__ b, int cout,
                                                  float* __restrict__ pre, float* __restrict__ post,
                                                  const float* __restrict__ r, const float* __restrict__ s,
                                                  float half_dt, float* __restrict__ z,
                                                  const float* __restrict__ gmul, int dil) {
    __shared__ float sw[kHid * kHid * 9];
    __shared__ float sb[kHid];
    const long long np = (long long)nx * nz;
    for (int i = threadIdx.x; i < cout * cin * 9; i += 256) sw[i] = W[i];
    for (int i = threadIdx.x; i < cout; i += 256) sb[i] = b ? b[i] : 0.0f;
    __syncthreads();
    const int lx = threadIdx.x & 63, lz = threadIdx.x >> 6;
    const int gx = blockIdx.x * kTX + lx, gz = blockIdx.y * kTZ + lz;
    if (gx >= nx || gz >= nz) return;
    float acc[kHid];
#pragma unroll
    for (int co = 0; co < kHid; ++co) acc[co] = co < cout ? sb[co] : 0.0f;
    for (int ci = 0; ci < cin; ++ci) {
        // inputs at the 9 dilated taps, read through the caches (zero outside the grid)
        float xv[9];
        const float inv_s = (MODE == L_FIRST) ? 1.0f / s[ci] : 1.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int xx = gx + dil * (t % 3 - 1), zz = gz + dil * (t / 3 - 1);
            float v = 0.0f;
            if (xx >= 0 && xx < nx && zz >= 0 && zz < nz) {
                const long long o = (long long)ci * np + (long long)zz * nx + xx;
                v = (MODE == L_FIRST) ? r[o] * inv_s : in[o];
            }
            xv[t] = v;
        }
#pragma unroll
        for (int co = 0; co < kHid; ++co) {
            if (co < cout) {
                const float* w = sw + (co * cin + ci) * 9;
                float a = acc[co];
#pragma unroll
                for (int t = 0; t < 9; ++t) a += w[t] * xv[t];
                acc[co] = a;
            }
        }
    }
    const long long o = (long long)gz * nx + gx;
#pragma unroll
    for (int co = 0; co < kHid; ++co) {
        if (co >= cout) continue;
        const float h = acc[co];
        if (MODE == L_LAST) {
            if (pre) pre[co * np + o] = h;
            if (z) z[co * np + o] = half_dt * r[co * np + o] + s[co] * h;
        } else {
            if (pre) pre[co * np + o] = h;
            if (post) post[co * np + o] = gmul ? h * gelu_grad(gmul[co * np + o]) : gelu(h);
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 MFMA convolution for inference.  Wave w of the block computes output row
// z0 + w, 64 pixels as four 16-pixel MFMA tiles; per tile 9 instructions
// (one per tap), A = 16 output x 16 input channels (the weights), B = 16 input
// channels x 16 pixels, FP32 accumulation.  Operand layout of
// v_mfma_f32_16x16x16_bf16: lane l holds A[row l%16][k 4(l/16)..+3],
// B[k 4(l/16)..+3][col l%16] and D[row 4(l/16)..+3][col l%16], so each lane
// ends with four consecutive output channels of one pixel: one 8-byte store.
// Wf: bf16 weights [tap][co][ci] padded to 16 x 16.
// ---------------------------------------------------------------------------
// Scale of the input, s = sqrt(mean r^2) over all fields (1 if r = 0), from
// per-block partial sums of squares (nsets sets of nblk), in the order
// k_field_scale adds them; every thread of the block gets it.
__device__ __forceinline__ float finish_scale(const double* __restrict__ partials, int nblk, int nsets, double count,
                                              double* red4, float* sh) {
    double tot = 0.0;
    for (int f = 0; f < nsets; ++f) tot += sum_partials(partials + (long long)f * nblk, nblk, 1, 0, red4);
    if (threadIdx.x == 0) {
        const double v = sqrt(tot / count);
        *sh = v > 0.0 ? (float)v : 1.0f;
    }
    __syncthreads();
    return *sh;
}

// Input scale per channel for the first layer: finished here from spart
// (block 0 stores it in s for the last layer) or read from s.
__device__ __forceinline__ void first_layer_scale(int cin, long long np, float* __restrict__ s,
                                                  const double* __restrict__ spart, int snblk, int snsets,
                                                  double* red, float* s_sh, float (&sc)[kHid]) {
    if (spart) {
        const float sv = finish_scale(spart, snblk, snsets, (double)np * cin, red, s_sh);
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < cin) s[threadIdx.x] = sv;
#pragma unroll
        for (int c = 0; c < kHid; ++c) sc[c] = sv;
    } else {
#pragma unroll
        for (int c = 0; c < kHid; ++c) sc[c] = c < cin ? s[c] : 1.0f;
    }
}

// Input tile of a layer, pixel-major with the channels innermost: rows
// z0 - h .. z0 + kTZ + h - 1 and columns x0 - h .. x0 + kTX + h - 1, zero
// outside the grid.  FIRST: the state vector r (channel-major FP32) divided by
// the scale and rounded to BF16, one pixel per thread and pass, its 16-channel
// row (zeros beyond cin) stored as two 16-byte halves; MID and LAST: hidden
// activations (pixel-major BF16, 32 bytes per pixel) copied as two 16-byte
// halves, four loads in flight per thread before their stores.
template <int MODE>
__device__ __forceinline__ void stage_input(int nx, int nz, int x0, int z0, int h,
                                            const unsigned short* __restrict__ in, int cin,
                                            const float* __restrict__ r, const float (&sc)[kHid],
                                            unsigned short* __restrict__ dst) {
    const long long np = (long long)nx * nz;
    const int SZ = kTZ + 2 * h, SX = kTX + 2 * h;
    if (MODE == L_FIRST) {
        for (int p = threadIdx.x; p < SZ * SX; p += 256) {
            const int lz = p / SX, lx = p - lz * SX;
            const int gx = x0 + lx - h, gz = z0 + lz - h;
            const bool inside = gx >= 0 && gx < nx && gz >= 0 && gz < nz;
            unsigned short hv[kHid];
#pragma unroll
            for (int c = 0; c < kHid; ++c) {
                hv[c] = 0;
                if (c < cin && inside) hv[c] = f2bf(r[(long long)c * np + (long long)gz * nx + gx] / sc[c]);
            }
            uint4 lo, hi;
            lo.x = hv[0] | ((unsigned)hv[1] << 16), lo.y = hv[2] | ((unsigned)hv[3] << 16);
            lo.z = hv[4] | ((unsigned)hv[5] << 16), lo.w = hv[6] | ((unsigned)hv[7] << 16);
            hi.x = hv[8] | ((unsigned)hv[9] << 16), hi.y = hv[10] | ((unsigned)hv[11] << 16);
            hi.z = hv[12] | ((unsigned)hv[13] << 16), hi.w = hv[14] | ((unsigned)hv[15] << 16);
            *reinterpret_cast<uint4*>(&dst[p * kHid]) = lo;
            *reinterpret_cast<uint4*>(&dst[p * kHid + 8]) = hi;
        }
    } else {
        const int nh = SZ * SX * 2;
        for (int i0 = threadIdx.x; i0 < nh; i0 += 4 * 256) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * 256, p = idx >> 1;
                const int lz = p / SX, lx = p - lz * SX;
                const int gx = x0 + lx - h, gz = z0 + lz - h;
                v[u] = uint4{0u, 0u, 0u, 0u};
                if (idx < nh && gx >= 0 && gx < nx && gz >= 0 && gz < nz)
                    v[u] = reinterpret_cast<const uint4*>(in + ((long long)gz * nx + gx) * kHid)[idx & 1];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * 256, p = idx >> 1;
                const int lz = p / SX, lx = p - lz * SX;
                if (idx < nh) *reinterpret_cast<uint4*>(&dst[(lz * SX + lx) * kHid + 8 * (idx & 1)]) = v[u];
            }
        }
    }
}

// A fragments of the 9 taps (weights): W[t][co = col][ci = 4 kg .. 4 kg + 3]
__device__ __forceinline__ void load_wfrag(const unsigned short* __restrict__ Wf, int col, int kg, bf16x4_t (&w)[9]) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const unsigned short* wp = Wf + ((t * kHid + col) * kHid + 4 * kg);
        w[t] = bf16x4_t{(short)wp[0], (short)wp[1], (short)wp[2], (short)wp[3]};
    }
}

// One 16-pixel subtile: the 9 dilated taps of a tile whose output pixel (row,
// px) sits at (row + dil, px + dil) of the staged input (stride SX pixels).
__device__ __forceinline__ f32x4_t conv_taps(const unsigned short* __restrict__ tile, int SX, int row, int px,
                                             int dil, const bf16x4_t (&w)[9], int kg) {
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int dz = (t / 3) * dil, dx = (t % 3) * dil;
        const bf16x4_t xv = *reinterpret_cast<const bf16x4_t*>(&tile[((row + dz) * SX + px + dx) * kHid + 4 * kg]);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[t], xv, acc, 0, 0, 0);
    }
    return acc;
}

// Output of one subtile at grid pixel pt: D[co = 4 kg + i][pixel = col] holds
// four consecutive output channels of one pixel.  MID: GELU, BF16, one 8-byte
// store (pixel-major); LAST: z = (dt/2) r + s (out), and z^2 added to zz.
template <int MODE>
__device__ __forceinline__ void layer_out(const f32x4_t& acc, const float (&bias)[4], int kg, int cout, long long np,
                                          long long pt, unsigned short* __restrict__ post,
                                          const float* __restrict__ r, const float* __restrict__ s, float half_dt,
                                          float* __restrict__ z, double& zz) {
    if (MODE == L_LAST) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = 4 * kg + i;
            if (co < cout) {
                const float zv = half_dt * r[co * np + pt] + s[co] * (acc[i] + bias[i]);
                z[co * np + pt] = zv;
                zz += (double)zv * zv;
            }
        }
    } else {
        u16x4_t o;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = f2bf(gelu_fast(acc[i] + bias[i]));
        *reinterpret_cast<u16x4_t*>(post + pt * kHid + 4 * kg) = o;
    }
}

// Optional fusions of the inference launches: with spart set, the first layer
// finishes the scale itself from per-block partial sums of r^2 (block 0 stores
// it in s for the last layer); with zpart set, the last layer leaves the
// block's partial sum of z^2 (the norm of the direction for the FD step of the
// next Jv) in zpart[block].
template <int MODE>
__global__ __launch_bounds__(256) void k_conv_mfma(int nx, int nz, const unsigned short* __restrict__ in, int cin,
                                                   const unsigned short* __restrict__ Wf,
                                                   const float* __restrict__ b, int cout,
                                                   unsigned short* __restrict__ post, const float* __restrict__ r,
                                                   float* __restrict__ s, float half_dt,
                                                   float* __restrict__ z, int dil, const double* __restrict__ spart,
                                                   int snblk, int snsets, double* __restrict__ zpart) {
    // staged input tile ((kTZ + 2 dil) x (kTX + 2 dil) pixels, sized by the launch)
    extern __shared__ __align__(16) unsigned short sin_[];
    __shared__ double red[4];
    __shared__ float s_sh;
    const long long np = (long long)nx * nz;
    const int x0 = blockIdx.x * kTX, z0 = blockIdx.y * kTZ;
    const int SX = kTX + 2 * dil;
    float sc[kHid];
    if (MODE == L_FIRST) first_layer_scale(cin, np, s, spart, snblk, snsets, red, &s_sh, sc);
    stage_input<MODE>(nx, nz, x0, z0, dil, in, cin, r, sc, sin_);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;          // k group of 4 channels
    bf16x4_t wfrag[9];
    load_wfrag(Wf, col, kg, wfrag);
    float bias[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = 4 * kg + i < cout ? b[4 * kg + i] : 0.0f;
    __syncthreads();
    const int gz = z0 + wv;
    double zz = 0.0;
    if (gz < nz) {
#pragma unroll
        for (int st = 0; st < kTX / 16; ++st) {
            const int px = st * 16 + col;                   // B column: pixel of this lane
            const f32x4_t acc = conv_taps(sin_, SX, wv, px, dil, wfrag, kg);
            const int gx = x0 + px;
            if (gx >= nx) continue;
            layer_out<MODE>(acc, bias, kg, cout, np, (long long)gz * nx + gx, post, r, s, half_dt, z, zz);
        }
    }
    if (MODE == L_LAST && zpart) {
        const double t = block_sum256(zz, red);
        if (threadIdx.x == 0) zpart[block_linear_id()] = t;
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// g = 2 (z - du) s / (||du||^2 B), and the partial loss sum (z - du)^2 / ||du||^2;
// a pair with du = 0 has no relative error and contributes nothing
__global__ __launch_bounds__(256) void k_loss_grad(const float* __restrict__ z, const float* __restrict__ du,
                                                   long long npts, int nf, const float* __restrict__ s,
                                                   const double* __restrict__ du2, double inv_batch,
                                                   float* __restrict__ g, double* __restrict__ partials) {
    __shared__ double red[4];
    const double nd2 = *du2;
    const double nd = nd2 > 0.0 ? nd2 : INFINITY;
    const long long n = npts * nf;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double d = (double)z[i] - (double)du[i];
        acc += d * d;
        const int f = (int)(i / npts);
        g[i] = (float)(2.0 * d * (double)s[f] / nd * inv_batch);
    }
    const double t = block_sum256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t / nd * inv_batch;
}

// Jacobian at rest J0 (acoustic-gravity terms about the hydrostatic background,
// closure off) and its transpose, FP32, one thread per point with the taps read
// through the caches under each field's own reflection parity:
//   (J0 v)_u = 2u/dt + theta0 Dx p         (J0^T y)_u = 2y_u/dt - Dx(kappa p_bar y_p)
//   (J0 v)_w = 2w/dt + theta0 Dz p         (J0^T y)_w = 2y_w/dt - Dz(kappa p_bar y_p)
//              - (g/theta0) theta                       + dp_bar/dz y_p + beta y_theta
//   (J0 v)_p = 2p/dt + dp_bar/dz w         (J0^T y)_p = 2y_p/dt - theta0 (Dx y_u + Dz y_w)
//              + kappa p_bar (Dx u + Dz w)
//   (J0 v)_theta = 2theta/dt + beta w      (J0^T y)_theta = 2y_theta/dt - (g/theta0) y_w
// (kappa p_bar y_p is formed at the source point of a reflected tap, i.e.
// extended like p).  partials[block] = sum of the squared outputs.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_rest_jac(Geo g, const float* __restrict__ in, float* __restrict__ out,
                                                  double* __restrict__ partials) {
    __shared__ double red[4];
    const long long np = g.npts;
    const int nx = g.nx, nz = g.nz;
    const bool perx = g.bcl == JFNK_BC_PERIODIC, perz = g.bcv == JFNK_BC_PERIODIC;
    const float ihx = (float)g.idx, ihz = (float)g.idz, tdt = (float)g.two_dt;
    const float th0 = (float)g.theta0, gth = (float)g.g_theta0, kap = (float)g.kappa, bet = (float)g.beta;
    const float* pb = g.pbar32;
    const float* dpb = g.dpbar32;
    // field f at the extended position (ex, ez), with its reflection sign; with
    // TRANS and f == 2 the product kappa p_bar y_p at the source point
    auto tap = [&](int f, int ex, int ez) -> float {
        int sx, sz;
        const int xs = s2d::map_axis(ex, nx, perx, sx);
        const int zs = s2d::map_axis(ez, nz, perz, sz);
        float v = in[(long long)f * np + (long long)zs * nx + xs];
        if (TRANS && f == 2) v *= kap * pb[zs];
        return s2d::sign2d(f, sx, sz, g.bcv) < 0 ? -v : v;
    };
    auto ddx = [&](int f, int x, int z) {
        return s2d::d5(tap(f, x - 2, z), tap(f, x - 1, z), tap(f, x + 1, z), tap(f, x + 2, z), ihx);
    };
    auto ddz = [&](int f, int x, int z) {
        return s2d::d5(tap(f, x, z - 2), tap(f, x, z - 1), tap(f, x, z + 1), tap(f, x, z + 2), ihz);
    };
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long long)gridDim.x * 256) {
        const int gz = (int)(i / nx), gx = (int)(i - (long long)gz * nx);
        const float u = in[i], w = in[np + i], p = in[2 * np + i], t = in[3 * np + i];
        float ou, ow, op, ot;
        if (!TRANS) {
            ou = tdt * u + th0 * ddx(2, gx, gz);
            ow = tdt * w + th0 * ddz(2, gx, gz) - gth * t;
            op = tdt * p + dpb[gz] * w + kap * pb[gz] * (ddx(0, gx, gz) + ddz(1, gx, gz));
            ot = tdt * t + bet * w;
        } else {
            ou = tdt * u - ddx(2, gx, gz);
            ow = tdt * w - ddz(2, gx, gz) + dpb[gz] * p + bet * t;
            op = tdt * p - th0 * (ddx(0, gx, gz) + ddz(1, gx, gz));
            ot = tdt * t - gth * w;
        }
        out[i] = ou;
        out[np + i] = ow;
        out[2 * np + i] = op;
        out[3 * np + i] = ot;
        acc += (double)ou * ou + (double)ow * ow + (double)op * op + (double)ot * ot;
    }
    const double tot = block_sum256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// e = z - du (elementwise)
__global__ __launch_bounds__(256) void k_sub(const float* __restrict__ a, const float* __restrict__ b, long long n,
                                             float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        out[i] = a[i] - b[i];
}

// loss (+)= sum(partials) / ||A du||^2 * inv_batch; g *= 2 s / (||A du||^2 B)
__global__ __launch_bounds__(256) void k_weighted_loss(const double* __restrict__ partials, int nblk,
                                                       const double* __restrict__ du2, double inv_batch,
                                                       double* __restrict__ loss, int accumulate) {
    __shared__ double red[4];
    const double t = sum_partials(partials, nblk, 1, 0, red);
    if (threadIdx.x == 0) {
        const double v = t / *du2 * inv_batch;
        *loss = accumulate ? *loss + v : v;
    }
}
__global__ __launch_bounds__(256) void k_scale_grad(float* __restrict__ g, long long npts, int nf,
                                                    const float* __restrict__ s, const double* __restrict__ du2,
                                                    double inv_batch) {
    const double c = 2.0 / *du2 * inv_batch;
    const long long n = npts * nf;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int f = (int)(i / npts);
        g[i] = (float)((double)g[i] * (double)s[f] * c);
    }
}

// dW[co][ci][t] and db[co] partial sums over one 64 x 4 tile of pixels; the
// input is staged one channel at a time with the halo of the layer's dilation
__global__ __launch_bounds__(256) void k_conv_wgrad(int nx, int nz, const float* __restrict__ g, int cout,
                                                    const float* __restrict__ a, int cin,
                                                    float* __restrict__ partials, int nw, int dil) {
    __shared__ float sg[kHid][kTZ][kTX];
    __shared__ float sa[kSZ][kSX];
    const long long np = (long long)nx * nz;
    const int x0 = blockIdx.x * kTX, z0 = blockIdx.y * kTZ;
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    float* out = partials + blk * (nw + cout);
    for (int idx = threadIdx.x; idx < cout * kTZ * kTX; idx += 256) {
        const int c = idx / (kTZ * kTX), rem = idx - c * (kTZ * kTX);
        const int lz = rem / kTX, lx = rem - lz * kTX;
        const int gx = x0 + lx, gz = z0 + lz;
        sg[c][lz][lx] = (gx < nx && gz < nz) ? g[(long long)c * np + (long long)gz * nx + gx] : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x < cout) {                        // bias gradient
        const int co = threadIdx.x;
        float acc = 0.0f;
        for (int lz = 0; lz < kTZ; ++lz)
            for (int lx = 0; lx < kTX; ++lx) acc += sg[co][lz][lx];
        out[nw + co] = acc;
    }
    const int SZ = kTZ + 2 * dil, SX = kTX + 2 * dil;
    for (int ci = 0; ci < cin; ++ci) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < SZ * SX; idx += 256) {
            const int lz = idx / SX, lx = idx - lz * SX;
            const int gx = x0 + lx - dil, gz = z0 + lz - dil;
            sa[lz][lx] = (gx >= 0 && gx < nx && gz >= 0 && gz < nz) ? a[(long long)ci * np + (long long)gz * nx + gx]
                                                                     : 0.0f;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < cout * 9; k += 256) {
            const int co = k / 9, t = k - co * 9;
            const int dz = (t / 3) * dil, dx = (t % 3) * dil;
            float acc = 0.0f;
            for (int lz = 0; lz < kTZ; ++lz)
                for (int lx = 0; lx < kTX; ++lx) acc += sg[co][lz][lx] * sa[lz + dz][lx + dx];
            out[(co * cin + ci) * 9 + t] = acc;
        }
    }
}

// grad[k] (+)= sum over blocks of partials[b][k] (fixed order, FP64)
__global__ __launch_bounds__(256) void k_wgrad_finish(const float* __restrict__ partials, int nblk, int cnt,
                                                      float* __restrict__ grad, int accumulate) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= cnt) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partials[(long long)b * cnt + k];
    grad[k] = accumulate ? grad[k] + (float)acc : (float)acc;
}

__global__ __launch_bounds__(256) void k_cast_scaled_input(const float* __restrict__ r, long long np, int nf,
                                                           const float* __restrict__ s, float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < np * nf) out[i] = r[i] / s[i / np];
}

// transposed, flipped weights for the backward-data convolution:
// Wt[ci][co][t] = W[co][ci][8 - t]; also the padded bf16 inference weights
// Wf[t][co][ci] (zero beyond cout / cin)
__global__ void k_prep_weights(const float* __restrict__ W, int cout, int cin, float* __restrict__ Wt,
                               unsigned short* __restrict__ Wf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cout * cin * 9) {
        const int co = k / (cin * 9), rem = k - co * (cin * 9);
        const int ci = rem / 9, t = rem - ci * 9;
        Wt[(ci * cout + co) * 9 + (8 - t)] = W[k];
    }
    if (k < 9 * kHid * kHid) {
        const int t = k / (kHid * kHid), rem = k - t * (kHid * kHid);
        const int co = rem / kHid, ci = rem - co * kHid;
        Wf[k] = (co < cout && ci < cin) ? f2bf(W[(co * cin + ci) * 9 + t]) : (unsigned short)0;
    }
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct NetLayer {
    int cin, cout, woff, boff;
};

static void layers_of(int nf, NetLayer L[4]) {
    const int ch[5] = {nf, kHid, kHid, kHid, nf};
    int o = 0;
    for (int l = 0; l < 4; ++l) {
        L[l].cin = ch[l];
        L[l].cout = ch[l + 1];
        L[l].woff = o;
        o += ch[l + 1] * ch[l] * 9;
        L[l].boff = o;
        o += ch[l + 1];
    }
}

int net_param_count(int nf) {
    NetLayer L[4];
    layers_of(nf, L);
    return L[3].boff + L[3].cout;
}

static dim3 tiles(int nx, int nz) { return dim3((nx + kTX - 1) / kTX, (nz + kTZ - 1) / kTZ); }

hipError_t net_prep_weights(const NetBuffers& nb, int nf, hipStream_t s) {
    NetLayer L[4];
    layers_of(nf, L);
    for (int l = 0; l < 4; ++l) {
        hipLaunchKernelGGL(k_prep_weights, dim3((9 * kHid * kHid + 255) / 256), dim3(256), 0, s, nb.theta + L[l].woff,
                           L[l].cout, L[l].cin, nb.wt + L[l].woff, nb.wbf + l * 9 * kHid * kHid);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int net_sumsq_blocks(long long np) {
    const int nblk = (int)std::min<long long>(512, (np + 1023) / 1024);
    return nblk < 1 ? 1 : nblk;
}

hipError_t net_field_sumsq(const float* r, long long np, int nf, double* partials, hipStream_t st) {
    hipLaunchKernelGGL(k_field_sumsq, dim3(net_sumsq_blocks(np), nf), dim3(256), 0, st, r, np, partials);
    return hipGetLastError();
}

hipError_t net_field_scale(const float* r, long long np, int nf, double* partials, float* s, hipStream_t st) {
    hipError_t e = net_field_sumsq(r, np, nf, partials, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_field_scale, dim3(1), dim3(256), 0, st, (const double*)partials, net_sumsq_blocks(np), nf,
                       (double)np * nf, nf, s);
    return hipGetLastError();
}

// The input scale for inference: from rpart (rnblk partial sums of r^2 over
// all fields, left by the producer of r) or from a pass over r.  Returns in
// (*part, *nblk, *nsets) the partials the first layer finishes itself, or
// part = null when a one-block launch has already written s.
hipError_t net_scale_source(const float* r, long long np, int nf, const double* rpart, int rnblk, double* partials,
                            float* s, int fuse_limit, const double** part, int* nblk, int* nsets, hipStream_t st) {
    *part = nullptr;
    if (rpart) {
        *nblk = rnblk;
        *nsets = 1;
    } else {
        hipError_t e = net_field_sumsq(r, np, nf, partials, st);
        if (e != hipSuccess) return e;
        *nblk = net_sumsq_blocks(np);
        *nsets = nf;
        rpart = partials;
    }
    if ((long long)(*nblk) * (*nsets) <= fuse_limit) {
        *part = rpart;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_field_scale, dim3(1), dim3(256), 0, st, rpart, *nblk, *nsets, (double)np * nf, nf, s);
    return hipGetLastError();
}

// inference: z = (dt/2) r + s N(r/s), BF16 MFMA (bf16 = true) or FP32.  In
// BF16 a problem with few scale partials has the scale finished inside the
// first layer; with ea set the last layer leaves the partial sums of ||z||^2
// and one finishing block forms the FD step of the next Jv.
hipError_t net_apply(const NetBuffers& nb, int nx, int nz, int nf, float half_dt, const float* r, float* z,
                     bool bf16, hipStream_t st, const EpsArgs* ea, const double* rpart, int rnblk) {
    NetLayer L[4];
    layers_of(nf, L);
    const dim3 grid = tiles(nx, nz);
    const long long np = (long long)nx * nz;
    if (bf16) {
        const double* spart = nullptr;
        int snblk = 0, snsets = 0;
        hipError_t e = net_scale_source(r, np, nf, rpart, rnblk, nb.partials, nb.s, kFuseScalePartials, &spart,
                                        &snblk, &snsets, st);
        if (e != hipSuccess) return e;
        unsigned short* a0 = nb.abf;
        unsigned short* a1 = nb.abf + kHid * np;
        auto lds = [](int d) { return (size_t)(kTZ + 2 * d) * (kTX + 2 * d) * kHid * sizeof(unsigned short); };
        constexpr int wl = 9 * kHid * kHid;   // bf16 weights per layer
        const double* none = nullptr;
        hipLaunchKernelGGL((k_conv_mfma<L_FIRST>), grid, dim3(256), lds(nb.dil[0]), st, nx, nz,
                           (const unsigned short*)nullptr, L[0].cin, nb.wbf + 0 * wl, nb.theta + L[0].boff, L[0].cout,
                           a0, r, nb.s, half_dt, (float*)nullptr, nb.dil[0], spart, snblk, snsets, (double*)nullptr);
        hipLaunchKernelGGL((k_conv_mfma<L_MID>), grid, dim3(256), lds(nb.dil[1]), st, nx, nz,
                           (const unsigned short*)a0, L[1].cin, nb.wbf + 1 * wl, nb.theta + L[1].boff, L[1].cout, a1,
                           r, nb.s, half_dt, (float*)nullptr, nb.dil[1], none, 0, 0, (double*)nullptr);
        hipLaunchKernelGGL((k_conv_mfma<L_MID>), grid, dim3(256), lds(nb.dil[2]), st, nx, nz,
                           (const unsigned short*)a1, L[2].cin, nb.wbf + 2 * wl, nb.theta + L[2].boff, L[2].cout, a0,
                           r, nb.s, half_dt, (float*)nullptr, nb.dil[2], none, 0, 0, (double*)nullptr);
        hipLaunchKernelGGL((k_conv_mfma<L_LAST>), grid, dim3(256), lds(nb.dil[3]), st, nx, nz,
                           (const unsigned short*)a0, L[3].cin, nb.wbf + 3 * wl, nb.theta + L[3].boff, L[3].cout,
                           (unsigned short*)nullptr, r, nb.s, half_dt, z, nb.dil[3], none, 0, 0,
                           ea ? ea->partials : (double*)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return ea ? launch_eps_finish((int)(grid.x * grid.y), *ea, st) : hipSuccess;
    }
    if (ea || rpart) return hipErrorInvalidValue;   // BF16 path only
    hipError_t e = net_field_scale(r, np, nf, nb.partials, nb.s, st);
    if (e != hipSuccess) return e;
    float* a0 = nb.act;                 // reuse the training buffers
    float* a1 = nb.act + kHid * np;
    hipLaunchKernelGGL((k_conv_f32<L_FIRST>), grid, dim3(256), 0, st, nx, nz, (const float*)nullptr, L[0].cin,
                       nb.theta + L[0].woff, nb.theta + L[0].boff, L[0].cout, (float*)nullptr, a0, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr, nb.dil[0]);
    hipLaunchKernelGGL((k_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, nz, (const float*)a0, L[1].cin,
                       nb.theta + L[1].woff, nb.theta + L[1].boff, L[1].cout, (float*)nullptr, a1, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr, nb.dil[1]);
    hipLaunchKernelGGL((k_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, nz, (const float*)a1, L[2].cin,
                       nb.theta + L[2].woff, nb.theta + L[2].boff, L[2].cout, (float*)nullptr, a0, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr, nb.dil[2]);
    hipLaunchKernelGGL((k_conv_f32<L_LAST>), grid, dim3(256), 0, st, nx, nz, (const float*)a0, L[3].cin,
                       nb.theta + L[3].woff, nb.theta + L[3].boff, L[3].cout, (float*)nullptr, (float*)nullptr, r,
                       nb.s, half_dt, z, (const float*)nullptr, nb.dil[3]);
    return hipGetLastError();
}

// loss and gradient (accumulated into nb.grad) of one pair, FP32 forward/backward;
// returns the loss contribution in nb.loss (device double, accumulated)
hipError_t net_pair_grad(const NetBuffers& nb, int nx, int nz, int nf, float half_dt, const float* r,
                         const float* du, double inv_batch, bool first_pair, const Geo& geo, hipStream_t st) {
    NetLayer L[4];
    layers_of(nf, L);
    const long long np = (long long)nx * nz;
    const dim3 grid = tiles(nx, nz);
    hipError_t e = net_field_scale(r, (long long)nx * nz, nf, nb.partials, nb.s, st);
    if (e != hipSuccess) return e;
    // forward, keeping pre-activations h_l and post-activations a_l
    float* act[4];
    float* pre[4];
    for (int l = 0; l < 4; ++l) {
        act[l] = nb.act + (long long)l * kHid * np;   // input of layer l+1 (a_{l+1})
        pre[l] = nb.pre + (long long)l * kHid * np;
    }
    hipLaunchKernelGGL((k_conv_f32<L_FIRST>), grid, dim3(256), 0, st, nx, nz, (const float*)nullptr, L[0].cin,
                       nb.theta + L[0].woff, nb.theta + L[0].boff, L[0].cout, pre[0], act[0], r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr, nb.dil[0]);
    for (int l = 1; l < 3; ++l)
        hipLaunchKernelGGL((k_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, nz, (const float*)act[l - 1], L[l].cin,
                           nb.theta + L[l].woff, nb.theta + L[l].boff, L[l].cout, pre[l], act[l], r, nb.s, half_dt,
                           (float*)nullptr, (const float*)nullptr, nb.dil[l]);
    hipLaunchKernelGGL((k_conv_f32<L_LAST>), grid, dim3(256), 0, st, nx, nz, (const float*)act[2], L[3].cin,
                       nb.theta + L[3].woff, nb.theta + L[3].boff, L[3].cout, pre[3], (float*)nullptr, r, nb.s,
                       half_dt, nb.z, (const float*)nullptr, nb.dil[3]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nb.loss_kind == NET_LOSS_REST_JACOBIAN) {
        // ||J0 du||^2; t = J0 (z - du) and its squared norm; g = J0^T t scaled
        const int nblk = (int)std::min<long long>(1024, (np + 255) / 256);
        float* ebuf = nb.g0;
        float* tbuf = nb.g1;
        hipLaunchKernelGGL(k_rest_jac<false>, dim3(nblk), dim3(256), 0, st, geo, du, tbuf, nb.partials);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_reduce_partials(nb.partials, nblk, 1, 1, nb.scal, 0, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_sub, dim3(nblk), dim3(256), 0, st, (const float*)nb.z, du, np * nf, ebuf);
        hipLaunchKernelGGL(k_rest_jac<false>, dim3(nblk), dim3(256), 0, st, geo, (const float*)ebuf, tbuf,
                           nb.partials + 4096);
        hipLaunchKernelGGL(k_weighted_loss, dim3(1), dim3(256), 0, st, (const double*)(nb.partials + 4096), nblk,
                           (const double*)nb.scal, inv_batch, nb.loss, first_pair ? 0 : 1);
        hipLaunchKernelGGL(k_rest_jac<true>, dim3(nblk), dim3(256), 0, st, geo, (const float*)tbuf, ebuf,
                           nb.partials);
        hipLaunchKernelGGL(k_scale_grad, dim3(nblk), dim3(256), 0, st, ebuf, np, nf, (const float*)nb.s,
                           (const double*)nb.scal, inv_batch);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        if ((e = net_solution_loss(nb, np, nf, du, inv_batch, first_pair, st)) != hipSuccess) return e;
    }
    // backward through the layers
    float* g = nb.g0;
    float* gnext = nb.g1;
    const int nt = (int)(grid.x * grid.y);
    for (int l = 3; l >= 0; --l) {
        const float* a_in = l == 0 ? nb.a0 : act[l - 1];
        if (l == 0) {
            // the scaled input r / s of the first layer
            if ((e = net_cast_scaled(r, np, nf, nb.s, nb.a0, st)) != hipSuccess) return e;
        }
        const int nw = L[l].cout * L[l].cin * 9;
        hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, st, nx, nz, (const float*)g, L[l].cout, a_in, L[l].cin,
                           nb.wpart, nw, nb.dil[l]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = net_wgrad_finish(nb.wpart, nt, nw + L[l].cout, nb.grad + L[l].woff, !first_pair, st)) !=
            hipSuccess)
            return e;
        if (l > 0) {
            // g_in = conv(g, W transposed and flipped) * gelu'(h_{l-1})
            hipLaunchKernelGGL((k_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, nz, (const float*)g, L[l].cout,
                               nb.wt + L[l].woff, (const float*)nullptr, L[l].cin, (float*)nullptr, gnext, r, nb.s,
                               half_dt, (float*)nullptr, (const float*)pre[l - 1], nb.dil[l]);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            std::swap(g, gnext);
        }
    }
    return hipSuccess;
}

// g0 = dL/d(network output) and the loss for the solution-space norm, from nb.z
hipError_t net_solution_loss(const NetBuffers& nb, long long np, int nf, const float* du, double inv_batch,
                             bool first_pair, hipStream_t st) {
    const long long n = np * nf;
    const int nblk = (int)std::max<long long>(1, std::min<long long>(1024, (n + 1023) / 1024));
    hipLaunchKernelGGL(k_field_sumsq, dim3(nblk, 1), dim3(256), 0, st, du, n, nb.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_reduce_partials(nb.partials, nblk, 1, 1, nb.scal, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_grad, dim3(nblk), dim3(256), 0, st, nb.z, du, np, nf, nb.s, nb.scal, inv_batch, nb.g0,
                       nb.partials + 4096);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_reduce_partials(nb.partials + 4096, nblk, 1, 1, nb.loss, first_pair ? 0 : 1, st);
}

hipError_t net_cast_scaled(const float* r, long long np, int nf, const float* s, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_scaled_input, dim3((unsigned)((np * nf + 255) / 256)), dim3(256), 0, st, r, np, nf, s,
                       out);
    return hipGetLastError();
}

hipError_t net_wgrad_finish(const float* partials, int nblk, int cnt, float* grad, bool accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_wgrad_finish, dim3((cnt + 255) / 256), dim3(256), 0, st, partials, nblk, cnt, grad,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t net_adam(const NetBuffers& nb, int n, int t, float lr, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, nb.theta, (const float*)nb.grad, nb.m, nb.v, n,
                       lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

}  // namespace jfnk
