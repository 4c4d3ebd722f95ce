// Learned right preconditioner for 3D problems: the network of the 2D path with
// 3 x 3 x 3 kernels (taps at (-1, 0, 1) along z, y and x, dilation 1):
//     z = (dt/2) r + s N(r / s),     s = RMS of r over all fields (1 if r = 0),
//     N = conv(nf->16) GELU conv(16->16) GELU conv(16->16) GELU conv(16->nf),
// zero padding, erf GELU.  Inference runs in BF16 on MFMA
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation, one tap per instruction, 27
// per 16-point subtile, erf by a rational approximation inside the BF16
// rounding); training (forward, backward, Adam) runs in FP32 with the exact erf.
//
// The FP32 training activations are channel-major [c][nz][ny][nx] like the
// state vectors; the BF16 inference activations are pixel-major [point][16].
// Parameters: one flat FP32 vector, per layer W[co][ci][kz][ky][kx] then b[co].

#include "jfnk_internal.hpp"
#include "reduce.hpp"

#include <algorithm>
#include <cmath>

namespace jfnk {

namespace {

constexpr int kHid = 16;
constexpr int kTaps = 27;
constexpr int kTX = 64, kTY = 4;      // output points per 256-thread block (one z plane)
constexpr int kWZ = 4;                // z planes per weight-gradient block
constexpr int kSX = kTX + 2, kSY = kTY + 2, kSZ = 3;
// the first layer finishes the input scale itself below this many partials
constexpr int kFuseScalePartials3 = 1024;

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {   // round to nearest even
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

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

__device__ __forceinline__ void tap_offsets(int t, int& dz, int& dy, int& dx) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// FP32 convolution, one thread per point, taps read through the caches
// FIRST: in = r / s;  MID: in = act;  LAST: z = (dt/2) r + s (out_pre)
// post = GELU(out_pre), or with gmul out_pre * gelu'(gmul) (backward data)
template <int MODE>
__global__ __launch_bounds__(256) void k3_conv_f32(int nx, int ny, int nz, const float* __restrict__ in, int cin,
                                                   const float* __restrict__ W, const float* __restrict__ b, int cout,
                                                   float* __restrict__ pre, float* __restrict__ post,
                                                   const float* __restrict__ r, const float* __restrict__ s,
                                                   float half_dt, float* __restrict__ z,
                                                   const float* __restrict__ gmul) {
    __shared__ float sw[kHid * kHid * kTaps];
    __shared__ float sb[kHid];
    const long long np = (long long)nx * ny * nz;
    for (int i = threadIdx.x; i < cout * cin * kTaps; i += 256) sw[i] = W[i];
    for (int i = threadIdx.x; i < cout; i += 256) sb[i] = b ? b[i] : 0.0f;
    __syncthreads();
    const int gx = blockIdx.x * kTX + (threadIdx.x & 63);
    const int gy = blockIdx.y * kTY + (threadIdx.x >> 6);
    const int gz = blockIdx.z;
    if (gx >= nx || gy >= ny) return;
    float acc[kHid];
#pragma unroll
    for (int co = 0; co < kHid; ++co) acc[co] = co < cout ? sb[co] : 0.0f;
    for (int ci = 0; ci < cin; ++ci) {
        const float inv_s = (MODE == L_FIRST) ? 1.0f / s[ci] : 1.0f;
        float xv[kTaps];
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            int dz, dy, dx;
            tap_offsets(t, dz, dy, dx);
            const int xx = gx + dx, yy = gy + dy, zz = gz + dz;
            float v = 0.0f;
            if (xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz) {
                const long long o = (long long)ci * np + ((long long)zz * ny + yy) * nx + xx;
                v = (MODE == L_FIRST) ? r[o] * inv_s : in[o];
            }
            xv[t] = v;
        }
#pragma unroll
        for (int co = 0; co < kHid; ++co) {
            if (co < cout) {
                const float* w = sw + (co * cin + ci) * kTaps;
                float a = acc[co];
#pragma unroll
                for (int t = 0; t < kTaps; ++t) a += w[t] * xv[t];
                acc[co] = a;
            }
        }
    }
    const long long o = ((long long)gz * ny + gy) * nx + gx;
#pragma unroll
    for (int co = 0; co < kHid; ++co) {
        if (co >= cout) continue;
        const float h = acc[co];
        if (pre) pre[co * np + o] = h;
        if (MODE == L_LAST) {
            if (z) z[co * np + o] = half_dt * r[co * np + o] + s[co] * h;
        } else if (post) {
            post[co * np + o] = gmul ? h * gelu_grad(gmul[co * np + o]) : gelu(h);
        }
    }
}

// BF16 3 x 3 x 3 convolution for inference, marching along z: a block of
// four waves owns 64 x 8 output points over a chunk of planes; the input
// planes z-1, z, z+1 over the tile grown by one sit in an LDS ring of three
// (pixel-major, 16 BF16 channels per point), and the next plane is loaded to
// registers while plane z is computed.  Each wave computes two output rows of
// four 16-point subtiles; a B fragment of an input row serves the taps of both
// rows that read it (four rows loaded per (dz, dx) instead of six).
// v_mfma_f32_16x16x16_bf16 with A = the weights of one tap (output x input
// channels) and B = input channels x 16 points, FP32 accumulation, so each
// lane ends with four consecutive output channels of one point.  FIRST: input
// r / s (channel-major FP32); MID, LAST: pixel-major BF16 activations.
// Optional fusions, as in the 2D network: spart (the first layer finishes the
// scale from per-block partial sums of r^2, block 0 stores it in s) and zpart
// (the last layer's per-block partial sum of z^2).
constexpr int kMX = 64, kMY = 8;                                    // output points per block and plane
constexpr int kMSX = kMX + 2, kMSY = kMY + 2, kMPL = kMSX * kMSY;   // staged plane: 660 points
constexpr int kMPT = (kMPL + 255) / 256;                            // staged points per thread (3)

template <int MODE>
__global__ __launch_bounds__(256) void k3_conv_march(int nx, int ny, int nz, const unsigned short* __restrict__ in,
                                                     int cin, const unsigned short* __restrict__ Wf,
                                                     const float* __restrict__ b, int cout,
                                                     unsigned short* __restrict__ post, const float* __restrict__ r,
                                                     float* __restrict__ s, float half_dt, float* __restrict__ z,
                                                     const double* __restrict__ spart, int snblk, int snsets,
                                                     double* __restrict__ zpart, int kzc) {
    __shared__ __align__(16) unsigned short ring[3][kMPL][kHid];
    __shared__ double red[4];
    __shared__ float s_sh;
    const long long np = (long long)nx * ny * nz;
    const int x0 = blockIdx.x * kMX, y0 = blockIdx.y * kMY;
    const int zc0 = blockIdx.z * kzc, zc1 = min(zc0 + kzc, nz);
    float sc = 1.0f;   // the input scale (FIRST)
    if (MODE == L_FIRST) {
        if (spart) {
            double tot = 0.0;
            for (int f = 0; f < snsets; ++f) tot += sum_partials(spart + (long long)f * snblk, snblk, 1, 0, red);
            if (threadIdx.x == 0) {
                const double v = sqrt(tot / ((double)np * cin));
                s_sh = v > 0.0 ? (float)v : 1.0f;
            }
            __syncthreads();
            sc = s_sh;
            if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x < cin) s[threadIdx.x] = sc;
        } else {
            sc = s[0];   // one scale for every field
        }
    }
    // the staged points of this thread: p = tid + 256 k
    int soff[kMPT];
    bool inside[kMPT];
#pragma unroll
    for (int k = 0; k < kMPT; ++k) {
        const int p = threadIdx.x + 256 * k;
        const int ly = p / kMSX, lx = p - ly * kMSX;
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        inside[k] = p < kMPL && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        soff[k] = inside[k] ? gy * nx + gx : 0;
    }
    // one plane's share of this thread into registers (zeros outside the
    // grid); FIRST keeps the raw FP32 values and converts them at the store,
    // so that the loads stay in flight under the compute of the plane before
    constexpr int kMaxIn = 8;   // input fields of the first layer (nf <= 8)
    uint4 st[kMPT][2];
    float rv[kMPT][kMaxIn];
    auto load_plane = [&](int zz) {
        const bool zin = zz >= 0 && zz < nz;
#pragma unroll
        for (int k = 0; k < kMPT; ++k) {
            const bool ok = zin && inside[k];
            const long long pt = (long long)zz * nx * ny + soff[k];
            if (MODE == L_FIRST) {
#pragma unroll
                for (int c = 0; c < kMaxIn; ++c) rv[k][c] = ok && c < cin ? r[(long long)c * np + pt] : 0.0f;
            } else {
                st[k][0] = uint4{0u, 0u, 0u, 0u};
                st[k][1] = uint4{0u, 0u, 0u, 0u};
                if (ok) {
                    const uint4* src = reinterpret_cast<const uint4*>(in + pt * kHid);
                    st[k][0] = src[0];
                    st[k][1] = src[1];
                }
            }
        }
    };
    auto store_plane = [&](int slot) {
#pragma unroll
        for (int k = 0; k < kMPT; ++k) {
            const int p = threadIdx.x + 256 * k;
            if (MODE == L_FIRST) {
                unsigned short hv[kMaxIn];
#pragma unroll
                for (int c = 0; c < kMaxIn; ++c) hv[c] = c < cin ? f2bf(rv[k][c] / sc) : 0;
                st[k][0] = uint4{hv[0] | ((unsigned)hv[1] << 16), hv[2] | ((unsigned)hv[3] << 16),
                                 hv[4] | ((unsigned)hv[5] << 16), hv[6] | ((unsigned)hv[7] << 16)};
                st[k][1] = uint4{0u, 0u, 0u, 0u};
            }
            if (p < kMPL) {
                *reinterpret_cast<uint4*>(&ring[slot][p][0]) = st[k][0];
                *reinterpret_cast<uint4*>(&ring[slot][p][8]) = st[k][1];
            }
        }
    };
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    bf16x4_t wfrag[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
        const unsigned short* wp = Wf + ((t * kHid + col) * kHid + 4 * kg);
        wfrag[t] = bf16x4_t{(short)wp[0], (short)wp[1], (short)wp[2], (short)wp[3]};
    }
    float bias[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = 4 * kg + i < cout ? b[4 * kg + i] : 0.0f;
    auto slot_of = [](int zz) { return (zz + 3) % 3; };   // zz >= -1
#pragma unroll 1
    for (int zz = zc0 - 1; zz <= zc0 + 1; ++zz) {
        load_plane(zz);
        store_plane(slot_of(zz));
    }
    __syncthreads();
    const int R0 = 2 * wv;   // this wave's output rows R0, R0 + 1 (staged rows R0 .. R0 + 3)
    double zz2 = 0.0;
    for (int zo = zc0; zo < zc1; ++zo) {
        const bool more = zo + 1 < zc1;
        if (more) load_plane(zo + 2);
        // LAST: r at this lane's outputs, loaded before the MFMAs
        float rr[2][4][4];
        if (MODE == L_LAST) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int gy = y0 + R0 + h, gx = x0 + q * 16 + col;
                    const long long pt = ((long long)zo * ny + gy) * nx + gx;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        rr[h][q][i] = gy < ny && gx < nx && 4 * kg + i < cout ? r[(4 * kg + i) * np + pt] : 0.0f;
                }
        }
        f32x4_t acc0[4], acc1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc0[q] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
            acc1[q] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const int sl = slot_of(zo - 1 + dz);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
                for (int yi = 0; yi < 4; ++yi) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bf16x4_t xv =
                            *reinterpret_cast<const bf16x4_t*>(&ring[sl][(R0 + yi) * kMSX + q * 16 + col + dx][4 * kg]);
                        if (yi <= 2)
                            acc0[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wfrag[dz * 9 + yi * 3 + dx], xv,
                                                                                 acc0[q], 0, 0, 0);
                        if (yi >= 1)
                            acc1[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wfrag[dz * 9 + (yi - 1) * 3 + dx],
                                                                                 xv, acc1[q], 0, 0, 0);
                    }
                }
            }
        }
        // D[co = 4 kg + i][point = col]: four consecutive output channels of one point
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gy = y0 + R0 + h;
            if (gy >= ny) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gx = x0 + q * 16 + col;
                if (gx >= nx) continue;
                const f32x4_t& acc = h == 0 ? acc0[q] : acc1[q];
                const long long pt = ((long long)zo * ny + gy) * nx + gx;
                if (MODE == L_LAST) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int co = 4 * kg + i;
                        if (co < cout) {
                            const float zv = half_dt * rr[h][q][i] + s[co] * (acc[i] + bias[i]);
                            z[co * np + pt] = zv;
                            zz2 += (double)zv * zv;
                        }
                    }
                } else {
                    u16x4_t o;
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = f2bf(gelu_fast(acc[i] + bias[i]));
                    *reinterpret_cast<u16x4_t*>(post + pt * kHid + 4 * kg) = o;
                }
            }
        }
        __syncthreads();   // every wave is done with plane zo - 1
        if (more) store_plane(slot_of(zo + 2));
        __syncthreads();
    }
    if (MODE == L_LAST && zpart) {
        const double t = block_sum256(zz2, red);
        if (threadIdx.x == 0)
            zpart[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
    }
}

// planes per block of the marching convolution: about two blocks per compute
// unit (256 CUs) at the largest grids, at least one plane
inline int march_kzc(int nx, int ny, int nz) {
    const long long cols = (long long)((nx + kMX - 1) / kMX) * ((ny + kMY - 1) / kMY);
    const long long want = (512 + cols - 1) / cols;
    const int kzc = (int)((nz + want - 1) / want);
    return kzc < 1 ? 1 : kzc;
}

// dW[co][ci][t] and db[co] partial sums over a 64 x 4 x kWZ block of points:
// per z plane the output gradient is staged once, the input one channel at a
// time (3 x 6 x 66 points); sums collect in LDS, one slot per thread.
__global__ __launch_bounds__(256) void k3_conv_wgrad(int nx, int ny, int nz, const float* __restrict__ g, int cout,
                                                     const float* __restrict__ a, int cin,
                                                     float* __restrict__ partials, int nw) {
    __shared__ float sg[kHid][kTY][kTX];
    __shared__ float sa[kSZ][kSY][kSX];
    __shared__ float sp[kHid * kHid * kTaps + kHid];
    const long long np = (long long)nx * ny * nz;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kWZ;
    const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    for (int k = threadIdx.x; k < nw + cout; k += 256) sp[k] = 0.0f;
    for (int pz = 0; pz < kWZ; ++pz) {
        const int gz = z0 + pz;
        if (gz >= nz) break;
        __syncthreads();
        for (int idx = threadIdx.x; idx < cout * kTY * kTX; idx += 256) {
            const int c = idx / (kTY * kTX), rem = idx - c * (kTY * kTX);
            const int ly = rem / kTX, lx = rem - ly * kTX;
            const int gx = x0 + lx, gy = y0 + ly;
            sg[c][ly][lx] = (gx < nx && gy < ny) ? g[(long long)c * np + ((long long)gz * ny + gy) * nx + gx] : 0.0f;
        }
        __syncthreads();
        if (threadIdx.x < cout) {
            float acc = 0.0f;
            for (int ly = 0; ly < kTY; ++ly)
                for (int lx = 0; lx < kTX; ++lx) acc += sg[threadIdx.x][ly][lx];
            sp[nw + threadIdx.x] += acc;
        }
        for (int ci = 0; ci < cin; ++ci) {
            __syncthreads();
            for (int idx = threadIdx.x; idx < kSZ * kSY * kSX; idx += 256) {
                const int lz = idx / (kSY * kSX), rem = idx - lz * (kSY * kSX);
                const int ly = rem / kSX, lx = rem - ly * kSX;
                const int gx = x0 + lx - 1, gy = y0 + ly - 1, zz = gz + lz - 1;
                sa[lz][ly][lx] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny && zz >= 0 && zz < nz)
                                     ? a[(long long)ci * np + ((long long)zz * ny + gy) * nx + gx]
                                     : 0.0f;
            }
            __syncthreads();
            for (int k = threadIdx.x; k < cout * kTaps; k += 256) {
                const int co = k / kTaps, t = k - co * kTaps;
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                float acc = 0.0f;
                for (int ly = 0; ly < kTY; ++ly)
                    for (int lx = 0; lx < kTX; ++lx) acc += sg[co][ly][lx] * sa[dz][ly + dy][lx + dx];
                sp[(co * cin + ci) * kTaps + t] += acc;
            }
        }
    }
    __syncthreads();
    float* out = partials + blk * (nw + cout);
    for (int k = threadIdx.x; k < nw + cout; k += 256) out[k] = sp[k];
}

// Wt[ci][co][26 - t] = W[co][ci][t] (transposed, flipped: backward data) and
// the padded bf16 inference weights Wf[t][co][ci]
__global__ void k3_prep_weights(const float* __restrict__ W, int cout, int cin, float* __restrict__ Wt,
                                unsigned short* __restrict__ Wf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cout * cin * kTaps) {
        const int co = k / (cin * kTaps), rem = k - co * (cin * kTaps);
        const int ci = rem / kTaps, t = rem - ci * kTaps;
        Wt[(ci * cout + co) * kTaps + (kTaps - 1 - t)] = W[k];
    }
    if (k < kTaps * kHid * kHid) {
        const int t = k / (kHid * kHid), rem = k - t * (kHid * kHid);
        const int co = rem / kHid, ci = rem - co * kHid;
        Wf[k] = (co < cout && ci < cin) ? f2bf(W[(co * cin + ci) * kTaps + t]) : (unsigned short)0;
    }
}

struct Layer3 {
    int cin, cout, woff, boff;
};

void layers3(int nf, Layer3 L[4]) {
    const int ch[5] = {nf, kHid, kHid, kHid, nf};
    int o = 0;
    for (int l = 0; l < 4; ++l) {
        L[l].cin = ch[l];
        L[l].cout = ch[l + 1];
        L[l].woff = o;
        o += ch[l + 1] * ch[l] * kTaps;
        L[l].boff = o;
        o += ch[l + 1];
    }
}

dim3 grid3(int nx, int ny, int nz) { return dim3((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY, nz); }

}  // namespace

int net3_param_count(int nf) {
    Layer3 L[4];
    layers3(nf, L);
    return L[3].boff + L[3].cout;
}

long long net3_wgrad_tiles(int nx, int ny, int nz) {
    return (long long)((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY) * ((nz + kWZ - 1) / kWZ);
}

hipError_t net3_prep_weights(const NetBuffers& nb, int nf, hipStream_t s) {
    Layer3 L[4];
    layers3(nf, L);
    for (int l = 0; l < 4; ++l) {
        hipLaunchKernelGGL(k3_prep_weights, dim3((kTaps * kHid * kHid + 255) / 256), dim3(256), 0, s,
                           nb.theta + L[l].woff, L[l].cout, L[l].cin, nb.wt + L[l].woff,
                           nb.wbf + l * kTaps * kHid * kHid);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t net3_apply(const NetBuffers& nb, int nx, int ny, int nz, int nf, float half_dt, const float* r, float* z,
                      bool bf16, hipStream_t st, const EpsArgs* ea, const double* rpart, int rnblk) {
    Layer3 L[4];
    layers3(nf, L);
    const long long np = (long long)nx * ny * nz;
    const dim3 grid = grid3(nx, ny, nz);
    if (bf16) {
        // the scale is finished inside the first layer on small grids (few
        // partials); with ea set the last layer leaves the partial sums of
        // ||z||^2 and one finishing block forms the FD step of the next Jv
        const double* spart = nullptr;
        int snblk = 0, snsets = 0;
        hipError_t e = net_scale_source(r, np, nf, rpart, rnblk, nb.partials, nb.s, kFuseScalePartials3, &spart,
                                        &snblk, &snsets, st);
        if (e != hipSuccess) return e;
        unsigned short* a0 = nb.abf;
        unsigned short* a1 = nb.abf + kHid * np;
        const int wl = kTaps * kHid * kHid;
        const double* none = nullptr;
        const int kzc = march_kzc(nx, ny, nz);
        const dim3 mgrid((nx + kMX - 1) / kMX, (ny + kMY - 1) / kMY, (nz + kzc - 1) / kzc);
        hipLaunchKernelGGL((k3_conv_march<L_FIRST>), mgrid, dim3(256), 0, st, nx, ny, nz,
                           (const unsigned short*)nullptr, L[0].cin, nb.wbf + 0 * wl, nb.theta + L[0].boff, L[0].cout,
                           a0, r, nb.s, half_dt, (float*)nullptr, spart, snblk, snsets, (double*)nullptr, kzc);
        hipLaunchKernelGGL((k3_conv_march<L_MID>), mgrid, dim3(256), 0, st, nx, ny, nz, (const unsigned short*)a0,
                           L[1].cin, nb.wbf + 1 * wl, nb.theta + L[1].boff, L[1].cout, a1, r, nb.s, half_dt,
                           (float*)nullptr, none, 0, 0, (double*)nullptr, kzc);
        hipLaunchKernelGGL((k3_conv_march<L_MID>), mgrid, dim3(256), 0, st, nx, ny, nz, (const unsigned short*)a1,
                           L[2].cin, nb.wbf + 2 * wl, nb.theta + L[2].boff, L[2].cout, a0, r, nb.s, half_dt,
                           (float*)nullptr, none, 0, 0, (double*)nullptr, kzc);
        hipLaunchKernelGGL((k3_conv_march<L_LAST>), mgrid, dim3(256), 0, st, nx, ny, nz, (const unsigned short*)a0,
                           L[3].cin, nb.wbf + 3 * wl, nb.theta + L[3].boff, L[3].cout, (unsigned short*)nullptr, r,
                           nb.s, half_dt, z, none, 0, 0, ea ? ea->partials : (double*)nullptr, kzc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return ea ? launch_eps_finish((int)(mgrid.x * mgrid.y * mgrid.z), *ea, st) : hipSuccess;
    }
    if (ea || rpart) return hipErrorInvalidValue;   // BF16 path only
    hipError_t e = net_field_scale(r, np, nf, nb.partials, nb.s, st);
    if (e != hipSuccess) return e;
    float* a0 = nb.act;
    float* a1 = nb.act + kHid * np;
    hipLaunchKernelGGL((k3_conv_f32<L_FIRST>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)nullptr, L[0].cin,
                       nb.theta + L[0].woff, nb.theta + L[0].boff, L[0].cout, (float*)nullptr, a0, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr);
    hipLaunchKernelGGL((k3_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)a0, L[1].cin,
                       nb.theta + L[1].woff, nb.theta + L[1].boff, L[1].cout, (float*)nullptr, a1, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr);
    hipLaunchKernelGGL((k3_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)a1, L[2].cin,
                       nb.theta + L[2].woff, nb.theta + L[2].boff, L[2].cout, (float*)nullptr, a0, r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr);
    hipLaunchKernelGGL((k3_conv_f32<L_LAST>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)a0, L[3].cin,
                       nb.theta + L[3].woff, nb.theta + L[3].boff, L[3].cout, (float*)nullptr, (float*)nullptr, r,
                       nb.s, half_dt, z, (const float*)nullptr);
    return hipGetLastError();
}

// Loss of one pair (solution-space norm) and its gradient, added into nb.grad
// unless first_pair.
hipError_t net3_pair_grad(const NetBuffers& nb, int nx, int ny, int nz, int nf, float half_dt, const float* r,
                          const float* du, double inv_batch, bool first_pair, hipStream_t st) {
    Layer3 L[4];
    layers3(nf, L);
    const long long np = (long long)nx * ny * nz;
    const dim3 grid = grid3(nx, ny, nz);
    hipError_t e = net_field_scale(r, np, nf, nb.partials, nb.s, st);
    if (e != hipSuccess) return e;
    float* act[4];
    float* pre[4];
    for (int l = 0; l < 4; ++l) {
        act[l] = nb.act + (long long)l * kHid * np;
        pre[l] = nb.pre + (long long)l * kHid * np;
    }
    hipLaunchKernelGGL((k3_conv_f32<L_FIRST>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)nullptr, L[0].cin,
                       nb.theta + L[0].woff, nb.theta + L[0].boff, L[0].cout, pre[0], act[0], r, nb.s, half_dt,
                       (float*)nullptr, (const float*)nullptr);
    for (int l = 1; l < 3; ++l)
        hipLaunchKernelGGL((k3_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)act[l - 1],
                           L[l].cin, nb.theta + L[l].woff, nb.theta + L[l].boff, L[l].cout, pre[l], act[l], r, nb.s,
                           half_dt, (float*)nullptr, (const float*)nullptr);
    hipLaunchKernelGGL((k3_conv_f32<L_LAST>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)act[2], L[3].cin,
                       nb.theta + L[3].woff, nb.theta + L[3].boff, L[3].cout, pre[3], (float*)nullptr, r, nb.s,
                       half_dt, nb.z, (const float*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = net_solution_loss(nb, np, nf, du, inv_batch, first_pair, st)) != hipSuccess) return e;
    float* g = nb.g0;
    float* gnext = nb.g1;
    const dim3 wgrid((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY, (nz + kWZ - 1) / kWZ);
    const int nt = (int)net3_wgrad_tiles(nx, ny, nz);
    for (int l = 3; l >= 0; --l) {
        const float* a_in = l == 0 ? nb.a0 : act[l - 1];
        if (l == 0 && (e = net_cast_scaled(r, np, nf, nb.s, nb.a0, st)) != hipSuccess) return e;
        const int nw = L[l].cout * L[l].cin * kTaps;
        hipLaunchKernelGGL(k3_conv_wgrad, wgrid, dim3(256), 0, st, nx, ny, nz, (const float*)g, L[l].cout, a_in,
                           L[l].cin, nb.wpart, nw);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = net_wgrad_finish(nb.wpart, nt, nw + L[l].cout, nb.grad + L[l].woff, !first_pair, st)) != hipSuccess)
            return e;
        if (l > 0) {
            // g_in = conv(g, W transposed and flipped) * gelu'(h_{l-1})
            hipLaunchKernelGGL((k3_conv_f32<L_MID>), grid, dim3(256), 0, st, nx, ny, nz, (const float*)g, L[l].cout,
                               nb.wt + L[l].woff, (const float*)nullptr, L[l].cin, (float*)nullptr, gnext, r, nb.s,
                               half_dt, (float*)nullptr, (const float*)pre[l - 1]);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            std::swap(g, gnext);
        }
    }
    return hipSuccess;
}

}  // namespace jfnk
