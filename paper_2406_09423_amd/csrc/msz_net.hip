// msz_net.hip -- the learned edit proposal: a 3-layer 3x3x3 conv net whose
// prediction warm-starts the correction loop (the loop still runs after it
// and judges).  BF16 weights and activations, FP32 accumulation, on MFMA.
//
// Parameters (FP32 master copy, one flat array, MSZ_NET_PARAMS floats):
//   W0[27][16][16] b0[16]      features (12 used, 16 stored) -> 16
//   W1[27][16][16] b1[16]      16 -> 16
//   W2[27][16]     b2[1]       16 -> 1
// tap = (dz+1)*9 + (dy+1)*3 + (dx+1); zero padding outside the grid.
// Activations: BF16, channel-last [vertex][16], vertex id x + nx*(y + ny*z).
//
// Convolution as GEMM on v_mfma_f32_16x16x32_bf16: M = 16 output channels,
// N = 16 x-consecutive vertices, K = 32 (tap, input channel) pairs per
// instruction.  A (weights) stays in registers for the whole kernel, B is a
// 16-byte read of 8 consecutive channels of one shifted vertex from the LDS
// input tile; a lane's result is 4 consecutive output channels of one vertex,
// written as one 8-byte store.
#include <cmath>
#include <cstring>
#include <vector>

#include "msz_internal.h"

namespace msz {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetC = 16;
constexpr int kOffW0 = 0, kOffB0 = kOffW0 + 27 * 16 * 16, kOffW1 = kOffB0 + 16, kOffB1 = kOffW1 + 27 * 16 * 16,
              kOffW2 = kOffB1 + 16, kOffB2 = kOffW2 + 27 * 16, kNetParams = kOffB2 + 1;
static_assert(kNetParams == MSZ_NET_PARAMS, "parameter layout");

// Conv tile: 16 (x) x TY x TZ output vertices, 256 threads = 4 waves.
template <int TY, int TZ>
struct ConvTile {
    static constexpr int X = 16, Y = TY, Z = TZ, HX = X + 2, HY = Y + 2, HZ = Z + 2;
    static constexpr int HALO = HX * HY * HZ;
    static constexpr int ROWS = Y * Z;  // x-rows of 16 vertices
};

__device__ __forceinline__ uint16_t bf16_bits(float v) {
    const __bf16 b = static_cast<__bf16>(v);  // round to nearest even
    return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_float(uint16_t u) { return __uint_as_float(static_cast<unsigned>(u) << 16); }

__device__ __forceinline__ void tap_delta(int tap, int& dx, int& dy, int& dz) {
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
}

// Weight source of one convolution launch: value(tap, in, out) =
//   W[(flip ? 26 - tap : tap) * s_tap + in * s_in + out * s_out]
// for in < n_in and out < n_out, zero otherwise (padding channels and taps).
struct WeightView {
    const float* W;
    const float* bias;  // n_out entries or nullptr
    int s_tap, s_in, s_out, n_in, n_out, flip;
};

__device__ __forceinline__ float weight_at(const WeightView& wv, int tap, int in, int out) {
    if (tap >= 27 || in >= wv.n_in || out >= wv.n_out) return 0.0f;
    const int t = wv.flip ? 26 - tap : tap;
    return wv.W[t * wv.s_tap + in * wv.s_in + out * wv.s_out];
}

// Loads the input tile t (16 x TY x TZ vertices plus a one-vertex halo, CH16
// 16-byte chunks per vertex, zeros outside the grid) into registers.
template <int TY, int TZ, int CH16, int PER>
__device__ __forceinline__ void conv_tile_load(const uint16_t* __restrict__ in, const Grid& gr, int t, int tx_n,
                                               int ty_n, uint4 (&buf)[PER]) {
    using T = ConvTile<TY, TZ>;
    constexpr int NCH = T::HALO * CH16;
    const int X0 = (t % tx_n) * T::X, Y0 = ((t / tx_n) % ty_n) * T::Y, Z0 = (t / (tx_n * ty_n)) * T::Z;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + 256 * k;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (e < NCH) {
            const int hv = e / CH16, ch = e - hv * CH16;
            const int hx = hv % T::HX, hy = (hv / T::HX) % T::HY, hz = hv / (T::HX * T::HY);
            const int x = X0 + hx - 1, y = Y0 + hy - 1, z = Z0 + hz - 1;
            if (x >= 0 && x < gr.nx && y >= 0 && y < gr.ny && z >= 0 && z < gr.nz) {
                const long vid = x + static_cast<long>(gr.nx) * y + static_cast<long>(gr.nxy) * z;
                v = reinterpret_cast<const uint4*>(in)[vid * CH16 + ch];
            }
        }
        buf[k] = v;
    }
}

enum : int { kConvHidden = 0, kConvFinal = 1, kConvBackData = 2 };

// out = conv(in) for CIN input channels stored per vertex.
//  kConvHidden:   out16[v][16] = bf16(relu(conv + bias))
//  kConvFinal:    out1[v]      = (conv + bias)[channel 0] (fp32, linear output)
//  kConvBackData: out16[v][16] = bf16(conv * (mask[v][c] > 0))  (gradient through ReLU)
template <int CIN, int TY, int TZ, int MODE>
__global__ void __launch_bounds__(256) k_conv(const uint16_t* __restrict__ in, Grid gr, WeightView wv,
                                              const uint16_t* __restrict__ mask, uint16_t* __restrict__ out16,
                                              float* __restrict__ out1) {
    using T = ConvTile<TY, TZ>;
    constexpr int KSTEPS = CIN == 16 ? 14 : 7;   // 27 taps (+1 zero tap) x CIN / 32
    constexpr int CH16 = CIN * 2 / 16;            // 16-byte chunks per vertex
    __shared__ uint4 tile[T::HALO * CH16];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;

    // A operand (weights) of every K step, in registers for the whole kernel
    bf16x8 wa[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int tap, ci;
            if (CIN == 16) {
                tap = 2 * s + (g >> 1);
                ci = 8 * (g & 1) + j;
            } else {
                tap = 4 * s + g;
                ci = j;
            }
            wa[s][j] = static_cast<__bf16>(weight_at(wv, tap, ci, m));
        }
    }
    float bias[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int co = 4 * g + i;
        bias[i] = (wv.bias && co < wv.n_out) ? wv.bias[co] : 0.0f;
    }

    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y, tz_n = (gr.nz + T::Z - 1) / T::Z;
    const int ntiles = tx_n * ty_n * tz_n;
    const ItemRange range = xcd_items(ntiles);
    // the input tile (with halo) of the next tile is loaded into registers
    // while the current one is computed from LDS
    constexpr int NCH = T::HALO * CH16;
    constexpr int PER = (NCH + 255) / 256;
    uint4 buf[PER];
    if (range.first < range.hi) conv_tile_load<TY, TZ, CH16, PER>(in, gr, range.first, tx_n, ty_n, buf);
    for (int t = range.first; t < range.hi; t += range.stride) {
        const int X0 = (t % tx_n) * T::X, Y0 = ((t / tx_n) % ty_n) * T::Y, Z0 = (t / (tx_n * ty_n)) * T::Z;
        __syncthreads();  // the previous tile's reads are done
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + 256 * k;
            if (e < NCH) tile[e] = buf[k];
        }
        __syncthreads();
        if (t + range.stride < range.hi) conv_tile_load<TY, TZ, CH16, PER>(in, gr, t + range.stride, tx_n, ty_n, buf);

        for (int row = wave; row < T::ROWS; row += 4) {
            const int ly = row % T::Y, lz = row / T::Y;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s) {
                int tap, chunk;
                if (CIN == 16) {
                    tap = 2 * s + (g >> 1);
                    chunk = g & 1;
                } else {
                    tap = 4 * s + g;
                    chunk = 0;
                }
                if (tap > 26) tap = 26;  // the zero-weight padding tap reads a valid address
                int dx, dy, dz;
                tap_delta(tap, dx, dy, dz);
                const int hv = (m + dx + 1) + T::HX * ((ly + dy + 1) + T::HY * (lz + dz + 1));
                const uint4 bv = tile[hv * CH16 + chunk];
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
            }
            const int x = X0 + m, y = Y0 + ly, z = Z0 + lz;
            if (x >= gr.nx || y >= gr.ny || z >= gr.nz) continue;
            const long vid = x + static_cast<long>(gr.nx) * y + static_cast<long>(gr.nxy) * z;
            if constexpr (MODE == kConvFinal) {
                if (g == 0) out1[vid] = acc[0] + bias[0];
            } else {
                uint16_t o[4];
                if constexpr (MODE == kConvHidden) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = bf16_bits(fmaxf(acc[i] + bias[i], 0.0f));
                } else {
                    const uint2 mk = reinterpret_cast<const uint2*>(mask)[vid * 4 + g];
                    const uint16_t mv[4] = {static_cast<uint16_t>(mk.x & 0xFFFFu), static_cast<uint16_t>(mk.x >> 16),
                                            static_cast<uint16_t>(mk.y & 0xFFFFu), static_cast<uint16_t>(mk.y >> 16)};
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = bf16_float(mv[i]) > 0.0f ? bf16_bits(acc[i]) : 0;
                }
                uint2 pk;
                pk.x = static_cast<unsigned>(o[0]) | (static_cast<unsigned>(o[1]) << 16);
                pk.y = static_cast<unsigned>(o[2]) | (static_cast<unsigned>(o[3]) << 16);
                reinterpret_cast<uint2*>(out16)[vid * 4 + g] = pk;
            }
        }
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// The output layer (16 -> 1 channels) with packed BF16 dot products on the
// VALU (v_dot2 accumulates two products into an FP32 sum): on the 16x16 MFMA
// tile it would use one of 16 output rows.  Same tile and halo staging as
// k_conv; a thread computes OPT x-consecutive outputs of one row, reading the
// OPT + 2 input columns of each (dy, dz) once.
template <int TY, int TZ>
__global__ void __launch_bounds__(256) k_conv_out(const uint16_t* __restrict__ in, Grid gr,
                                                  const float* __restrict__ W2, const float* __restrict__ b2,
                                                  float* __restrict__ out1) {
    using T = ConvTile<TY, TZ>;
    constexpr int CH16 = 2;
    constexpr int OPT = 16 * T::ROWS / 256;  // outputs per thread: 4 for 8 x 8 rows, 2 for 32 x 1
    constexpr int GX = 16 / OPT;             // threads per row
    static_assert(OPT * 256 == 16 * T::ROWS, "every output has one thread");
    __shared__ uint4 tile[T::HALO * CH16];
    __shared__ unsigned wpk[27 * 8];  // BF16 weight pairs (channels 2p, 2p + 1) of every tap
    for (int e = threadIdx.x; e < 27 * 8; e += 256) {
        const int tap = e / 8, q = e % 8;
        wpk[e] = static_cast<unsigned>(bf16_bits(W2[tap * 16 + 2 * q])) |
                 (static_cast<unsigned>(bf16_bits(W2[tap * 16 + 2 * q + 1])) << 16);
    }
    const float bias = b2[0];
    const int xg = threadIdx.x % GX, row = threadIdx.x / GX;
    const int ly = row % T::Y, lz = row / T::Y;

    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y, tz_n = (gr.nz + T::Z - 1) / T::Z;
    const ItemRange range = xcd_items(tx_n * ty_n * tz_n);
    constexpr int NCH = T::HALO * CH16;
    constexpr int PER = (NCH + 255) / 256;
    uint4 buf[PER];
    if (range.first < range.hi) conv_tile_load<TY, TZ, CH16, PER>(in, gr, range.first, tx_n, ty_n, buf);
    for (int t = range.first; t < range.hi; t += range.stride) {
        const int X0 = (t % tx_n) * T::X, Y0 = ((t / tx_n) % ty_n) * T::Y, Z0 = (t / (tx_n * ty_n)) * T::Z;
        __syncthreads();  // the previous tile's reads (and the weight packing) are done
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + 256 * k;
            if (e < NCH) tile[e] = buf[k];
        }
        __syncthreads();
        if (t + range.stride < range.hi) conv_tile_load<TY, TZ, CH16, PER>(in, gr, t + range.stride, tx_n, ty_n, buf);
        float acc[OPT];
#pragma unroll
        for (int i = 0; i < OPT; ++i) acc[i] = bias;
        // one (dy, dz) row group at a time keeps OPT + 2 columns live
#pragma unroll 1
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll 1
            for (int dy = -1; dy <= 1; ++dy) {
                unsigned col[OPT + 2][8];
#pragma unroll
                for (int c = 0; c < OPT + 2; ++c) {
                    const int hv = (xg * OPT + c) + T::HX * ((ly + dy + 1) + T::HY * (lz + dz + 1));
                    const uint4 u0 = tile[hv * CH16], u1 = tile[hv * CH16 + 1];
                    col[c][0] = u0.x, col[c][1] = u0.y, col[c][2] = u0.z, col[c][3] = u0.w;
                    col[c][4] = u1.x, col[c][5] = u1.y, col[c][6] = u1.z, col[c][7] = u1.w;
                }
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    unsigned w[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) w[q] = wpk[tap * 8 + q];
#pragma unroll
                    for (int i = 0; i < OPT; ++i)
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            acc[i] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, col[i + dx + 1][q]),
                                                                     __builtin_bit_cast(bf16x2, w[q]), acc[i], false);
                }
            }
        const int y = Y0 + ly, z = Z0 + lz;
        if (y < gr.ny && z < gr.nz) {
#pragma unroll
            for (int i = 0; i < OPT; ++i) {
                const int x = X0 + xg * OPT + i;
                if (x < gr.nx) out1[x + static_cast<long>(gr.nx) * y + static_cast<long>(gr.nxy) * z] = acc[i];
            }
        }
    }
}

// Weight gradient of one layer, one partial sum per tile:
//   part[tile][tap][ci][co] = sum over the tile's vertices v of in[v + tap][ci] * dz[v][co]
//   part_b[tile][co]        = sum over the tile's vertices v of dz[v][co]
// M = 16 input channels, N = 16 output channels, K = 32 vertices per MFMA.
template <int CIN, int TY, int TZ>
__global__ void __launch_bounds__(256) k_conv_dw(const uint16_t* __restrict__ in, const uint16_t* __restrict__ dz,
                                                 Grid gr, float* __restrict__ part, float* __restrict__ part_b) {
    using T = ConvTile<TY, TZ>;
    constexpr int NV = T::X * T::ROWS;
    __shared__ uint16_t sin[T::HALO * CIN];
    __shared__ uint16_t sdz[NV * kNetC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int tile = blockIdx.x;
    const int X0 = (tile % tx_n) * T::X, Y0 = ((tile / tx_n) % ty_n) * T::Y, Z0 = (tile / (tx_n * ty_n)) * T::Z;
    constexpr int CH16 = CIN * 2 / 16;
    for (int e = threadIdx.x; e < T::HALO * CH16; e += 256) {
        const int hv = e / CH16, ch = e - hv * CH16;
        const int hx = hv % T::HX, hy = (hv / T::HX) % T::HY, hz = hv / (T::HX * T::HY);
        const int x = X0 + hx - 1, y = Y0 + hy - 1, z = Z0 + hz - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (x >= 0 && x < gr.nx && y >= 0 && y < gr.ny && z >= 0 && z < gr.nz)
            v = reinterpret_cast<const uint4*>(in)[(x + static_cast<long>(gr.nx) * y + static_cast<long>(gr.nxy) * z) * CH16 + ch];
        reinterpret_cast<uint4*>(sin)[e] = v;
    }
    for (int e = threadIdx.x; e < NV * 2; e += 256) {
        const int lv = e >> 1, ch = e & 1;
        const int x = X0 + lv % T::X, r = lv / T::X, y = Y0 + r % T::Y, z = Z0 + r / T::Y;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);  // vertices outside the grid contribute nothing
        if (x < gr.nx && y < gr.ny && z < gr.nz)
            v = reinterpret_cast<const uint4*>(dz)[(x + static_cast<long>(gr.nx) * y + static_cast<long>(gr.nxy) * z) * 2 + ch];
        reinterpret_cast<uint4*>(sdz)[e] = v;
    }
    __syncthreads();
    for (int tap = wave; tap < 27; tap += 4) {
        int dx, dy, dzz;
        tap_delta(tap, dx, dy, dzz);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < NV / 32; ++ks) {
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int lv = 32 * ks + 8 * g + j;  // output vertex of the tile
                const int lx = lv % T::X, r = lv / T::X, ly = r % T::Y, lz = r / T::Y;
                const int hv = (lx + dx + 1) + T::HX * ((ly + dy + 1) + T::HY * (lz + dzz + 1));
                a[j] = m < CIN ? __builtin_bit_cast(__bf16, sin[hv * CIN + (m < CIN ? m : 0)]) : static_cast<__bf16>(0.0f);
                b[j] = __builtin_bit_cast(__bf16, sdz[lv * kNetC + m]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        // acc[i] = D[ci = 4g + i][co = m]
        float* dst = part + (static_cast<long>(tile) * 27 + tap) * 16 * 16;
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[(4 * g + i) * 16 + m] = acc[i];
    }
    if (threadIdx.x < 16) {
        float sb = 0.0f;
        for (int lv = 0; lv < NV; ++lv) sb += bf16_float(sdz[lv * kNetC + threadIdx.x]);
        part_b[static_cast<long>(tile) * 16 + threadIdx.x] = sb;
    }
}

// Sums the per-tile partials into the gradient of one layer's weights and bias,
// in the parameter layout (out channels beyond n_out and in channels beyond
// n_in are dropped).
__global__ void __launch_bounds__(256) k_reduce_dw(const float* __restrict__ part, const float* __restrict__ part_b,
                                                   int ntiles, int n_in, int n_out, int s_in, float* __restrict__ gW,
                                                   float* __restrict__ gb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 27 * 16 * 16) {
        const int tap = e / 256, ci = (e / 16) % 16, co = e % 16;
        if (ci < n_in && co < n_out) {
            float s = 0.0f;
            for (int t = 0; t < ntiles; ++t) s += part[static_cast<long>(t) * 27 * 256 + e];
            gW[tap * n_in * s_in + ci * s_in + co] = s;
        }
    } else if (e < 27 * 256 + 16) {
        const int co = e - 27 * 256;
        if (co < n_out) {
            float s = 0.0f;
            for (int t = 0; t < ntiles; ++t) s += part_b[static_cast<long>(t) * 16 + co];
            gb[co] = s;
        }
    }
}

// Input channels of the net (16 stored per vertex, 12 used; the box is the
// 3x3x3 block around the vertex clipped to the grid, the clamps are [-8, 8]):
//   0 (fhat - box mean of fhat) / xi     1 log10(xi / value range) / 4 + 1
//   2..5 FPmax, FPmin, FNmax, FNmin of fhat against f
//   6 (fhat - f) / xi                    7 (f - box mean of f) / xi
//   8 dn_f(u) = i for an FPmin neighbour u       9 up_fhat(u) = i for an FNmax neighbour u
//   10 dn_f(u) = i for a neighbour u with dn_fhat(u) != dn_f(u)
//   11 up_fhat(u) = i for a neighbour u with up_fhat(u) != up_f(u)
// Channels 8..11 gather over the neighbour slots: neighbour j = i + off[s]
// points back at i through the opposite slot s ^ 1.
// One thread per (x, y) column walks z, keeping the 3x3 in-plane sums of f
// and fhat and the 3x3 direction bytes of planes z - 1, z, z + 1, so every
// plane is read once per column (36 loads per vertex instead of 82).  A
// direction byte of 0 stands for "outside the grid": no in-grid vertex has
// its ascent and its descent in the same slot 0.
struct PlaneBox {
    double sf, sh;         // sums over the in-grid part of the 3x3 block
    int cnt;               // its in-grid vertices
    unsigned wf[3], wh[3];  // row dy + 1: direction bytes of dx = -1, 0, 1 in bytes 0..2
    __device__ __forceinline__ unsigned df(int dx, int dy) const { return (wf[dy + 1] >> (8 * (dx + 1))) & 0xFFu; }
    __device__ __forceinline__ unsigned dh(int dx, int dy) const { return (wh[dy + 1] >> (8 * (dx + 1))) & 0xFFu; }
};

__device__ __forceinline__ PlaneBox load_plane_box(const float* __restrict__ f, const float* __restrict__ fhat,
                                                   const uint8_t* __restrict__ dirs_f,
                                                   const uint8_t* __restrict__ dirs_h, const Grid& gr, int x, int y,
                                                   int z) {
    PlaneBox P;
    P.sf = 0.0;
    P.sh = 0.0;
    P.cnt = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        P.wf[r] = 0u;
        P.wh[r] = 0u;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int xx = x + q - 1, yy = y + r - 1;
            if (z >= 0 && z < gr.nz && xx >= 0 && xx < gr.nx && yy >= 0 && yy < gr.ny) {
                const long j = xx + static_cast<long>(gr.nx) * yy + static_cast<long>(gr.nxy) * z;
                P.sf += f[j];
                P.sh += fhat[j];
                P.cnt += 1;
                P.wf[r] |= static_cast<unsigned>(dirs_f[j]) << (8 * q);
                P.wh[r] |= static_cast<unsigned>(dirs_h[j]) << (8 * q);
            }
        }
    }
    return P;
}

// Channels 8..11 of vertex i from the neighbour j in slot sl (plane Q).
__device__ __forceinline__ unsigned target_bits(const PlaneBox& Q, int sl, int dx, int dy) {
    const unsigned back = static_cast<unsigned>(sl ^ 1);
    const unsigned fj = Q.df(dx, dy), hj = Q.dh(dx, dy);
    const unsigned ufj = fj >> 4, nfj = fj & 15u, uhj = hj >> 4, nhj = hj & 15u;
    unsigned tg = 0;
    if (nhj == kSelf && nfj == back) tg |= 1u;  // FPmin at j targets dn_f(j)
    if (ufj == kSelf && uhj == back) tg |= 2u;  // FNmax at j targets up_fhat(j)
    if (nhj != nfj && nfj == back) tg |= 4u;
    if (uhj != ufj && uhj == back) tg |= 8u;
    return tg;
}

__global__ void __launch_bounds__(256) k_features(const float* __restrict__ f, const float* __restrict__ fhat,
                                                  const uint8_t* __restrict__ dirs_f,
                                                  const uint8_t* __restrict__ dirs_h, Grid gr, float xi, float xi_ch,
                                                  uint16_t* __restrict__ feat) {
    const unsigned one = bf16_bits(1.0f);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < gr.nxy; c += gridDim.x * blockDim.x) {
        const int x = c % gr.nx, y = c / gr.nx;
        PlaneBox pm = load_plane_box(f, fhat, dirs_f, dirs_h, gr, x, y, -1);  // plane z - 1
        PlaneBox p0 = load_plane_box(f, fhat, dirs_f, dirs_h, gr, x, y, 0);   // plane z
        for (int z = 0; z < gr.nz; ++z) {
            const PlaneBox pp = load_plane_box(f, fhat, dirs_f, dirs_h, gr, x, y, z + 1);  // plane z + 1
            const long i = c + static_cast<long>(gr.nxy) * z;
            const double sh = pm.sh + p0.sh + pp.sh, sf = pm.sf + p0.sf + pp.sf;
            const int n = pm.cnt + p0.cnt + pp.cnt;
            const double hi = fhat[i], fi = f[i];
            const float ch0 = fminf(fmaxf(static_cast<float>((hi - sh / n) / xi), -8.0f), 8.0f);
            const float ch6 = fminf(fmaxf(static_cast<float>((hi - fi) / xi), -8.0f), 8.0f);
            const float ch7 = fminf(fmaxf(static_cast<float>((fi - sf / n) / xi), -8.0f), 8.0f);
            const unsigned df = p0.df(0, 0), dh = p0.dh(0, 0);
            const unsigned uf = df >> 4, nf = df & 15u, uh = dh >> 4, nh = dh & 15u;
            const float fl[4] = {static_cast<float>((uh == kSelf) & (uf != kSelf)), static_cast<float>((nh == kSelf) & (nf != kSelf)),
                                 static_cast<float>((uf == kSelf) & (uh != kSelf)), static_cast<float>((nf == kSelf) & (nh != kSelf))};
            // the neighbour slots (offsets as in the slot table): in-plane ones, then the off-plane ones in 3D
            unsigned tg = target_bits(p0, 0, 1, 0) | target_bits(p0, 1, -1, 0) | target_bits(p0, 2, 0, 1) |
                          target_bits(p0, 3, 0, -1) | target_bits(p0, 4, 1, 1) | target_bits(p0, 5, -1, -1);
            if (gr.ndim == 3)
                tg |= target_bits(pp, 6, 0, 0) | target_bits(pm, 7, 0, 0) | target_bits(pp, 8, 1, 0) |
                      target_bits(pm, 9, -1, 0) | target_bits(pp, 10, 0, 1) | target_bits(pm, 11, 0, -1) |
                      target_bits(pp, 12, 1, 1) | target_bits(pm, 13, -1, -1);
            uint4 o0, o1;
            o0.x = static_cast<unsigned>(bf16_bits(ch0)) | (static_cast<unsigned>(bf16_bits(xi_ch)) << 16);
            o0.y = static_cast<unsigned>(bf16_bits(fl[0])) | (static_cast<unsigned>(bf16_bits(fl[1])) << 16);
            o0.z = static_cast<unsigned>(bf16_bits(fl[2])) | (static_cast<unsigned>(bf16_bits(fl[3])) << 16);
            o0.w = static_cast<unsigned>(bf16_bits(ch6)) | (static_cast<unsigned>(bf16_bits(ch7)) << 16);
            o1.x = ((tg & 1u) ? one : 0u) | (((tg & 2u) ? one : 0u) << 16);
            o1.y = ((tg & 4u) ? one : 0u) | (((tg & 8u) ? one : 0u) << 16);
            o1.z = 0u;
            o1.w = 0u;
            uint4* dst = reinterpret_cast<uint4*>(feat) + 2 * i;
            dst[0] = o0;
            dst[1] = o1;
            pm = p0;
            p0 = pp;
        }
    }
}

// Mean squared error: loss partial sums and dL/dp (the output layer is
// linear), stored as a 16-channel gradient tensor with channel 0 in use.
// Vertex i weighs 1 + edit_weight when its target is positive.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ p, const float* __restrict__ target, int n,
                                             float edit_weight, uint16_t* __restrict__ dz,
                                             float* __restrict__ loss_part) {
    __shared__ float red[4];
    float acc = 0.0f;
    const float scale = 2.0f / static_cast<float>(n);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float t = target[i];
        const float d = p[i] - t;
        const float w = t > 0.0f ? 1.0f + edit_weight : 1.0f;
        acc += w * d * d;
        const float gz = scale * w * d;
        uint4* row = reinterpret_cast<uint4*>(dz) + 2 * static_cast<long>(i);
        row[0] = make_uint4(bf16_bits(gz), 0u, 0u, 0u);
        row[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Adam (bias-corrected), FP32 master parameters.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, const float* __restrict__ grad,
                                              float* __restrict__ m1, float* __restrict__ m2, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float a = b1 * m1[i] + (1.0f - b1) * g;
        const float b = b2 * m2[i] + (1.0f - b2) * g * g;
        m1[i] = a;
        m2[i] = b;
        w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

// One decreasing edit (Eqs. 2-6 with the float floor L): halfway to the
// floor, snapped to it when float32 rounding would leave g unchanged.
__device__ __forceinline__ float halve_to(float g, float L) {
    const float h = __fmul_rn(__fadd_rn(g, L), 0.5f);
    return h == g ? L : h;
}

// Warm start: fhat halved k times, k = floor(fl(p - p_min)) + 1 clamped to
// [0, kMaxWarmHalvings] (0 where p is not a number).
constexpr int kMaxWarmHalvings = 64;
__global__ void __launch_bounds__(256) k_warm_start(const float* __restrict__ p, const float* __restrict__ L,
                                                    const float* __restrict__ fhat, float p_min, int n,
                                                    float* __restrict__ g0) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float q = floorf(__fsub_rn(p[i], p_min)) + 1.0f;
        const int k = q > 0.0f ? (q < static_cast<float>(kMaxWarmHalvings) ? static_cast<int>(q) : kMaxWarmHalvings) : 0;
        float g = fhat[i];
        if (k > 0) {
            const float l = L[i];
            for (int j = 0; j < k; ++j) g = halve_to(g, l);
        }
        g0[i] = g;
    }
}

// Training target: the number of halvings that take fhat_i to g_i (-1 when
// g_i is not on that chain within kMaxCount steps).
constexpr int kMaxCount = 256;
__global__ void __launch_bounds__(256) k_halvings(const float* __restrict__ L, const float* __restrict__ fhat,
                                                  const float* __restrict__ g, int n, float* __restrict__ k_out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i], l = L[i];
        float cur = fhat[i];
        int k = 0;
        while (cur > gi && k < kMaxCount) {
            const float nx = halve_to(cur, l);
            if (!(nx < cur)) break;  // at the floor (or an invalid floor): no further progress
            cur = nx;
            ++k;
        }
        k_out[i] = cur == gi ? static_cast<float>(k) : -1.0f;
    }
}

// ------------------------------------------------------------- launchers ---

constexpr int kConvBlocks = 2048;

template <int CIN, int MODE>
static void launch_conv_t(const uint16_t* in, const Grid& gr, const WeightView& wv, const uint16_t* mask,
                          uint16_t* out16, float* out1, hipStream_t s) {
    if (gr.nz == 1) {
        using T = ConvTile<32, 1>;
        const int nt = ((gr.nx + 15) / 16) * ((gr.ny + T::Y - 1) / T::Y) * gr.nz;
        hipLaunchKernelGGL((k_conv<CIN, 32, 1, MODE>), dim3(nt < kConvBlocks ? nt : kConvBlocks), dim3(256), 0, s, in, gr, wv,
                           mask, out16, out1);
    } else {
        using T = ConvTile<8, 8>;
        const int nt = ((gr.nx + 15) / 16) * ((gr.ny + T::Y - 1) / T::Y) * ((gr.nz + T::Z - 1) / T::Z);
        hipLaunchKernelGGL((k_conv<CIN, 8, 8, MODE>), dim3(nt < kConvBlocks ? nt : kConvBlocks), dim3(256), 0, s, in, gr, wv,
                           mask, out16, out1);
    }
}

static int conv_tiles(const Grid& gr) {
    if (gr.nz == 1) return ((gr.nx + 15) / 16) * ((gr.ny + 31) / 32);
    return ((gr.nx + 15) / 16) * ((gr.ny + 7) / 8) * ((gr.nz + 7) / 8);
}

template <int CIN>
static void launch_dw_t(const uint16_t* in, const uint16_t* dz, const Grid& gr, float* part, float* part_b,
                        hipStream_t s) {
    const int nt = conv_tiles(gr);
    if (gr.nz == 1) hipLaunchKernelGGL((k_conv_dw<CIN, 32, 1>), dim3(nt), dim3(256), 0, s, in, dz, gr, part, part_b);
    else hipLaunchKernelGGL((k_conv_dw<CIN, 8, 8>), dim3(nt), dim3(256), 0, s, in, dz, gr, part, part_b);
}

}  // namespace msz

// ================================================================ C ABI ====

namespace msz {
namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }
bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Net workspace of one field.
struct NetLayout {
    size_t dirs_f, dirs_h, feat, a1, a2, p, dz_a, dz_b, part, part_b, minmax, L, g0, total;
};

int conv_tile_count(const Grid& gr) { return conv_tiles(gr); }

NetLayout net_layout(const Grid& gr) {
    const size_t n = static_cast<size_t>(gr.n);
    const size_t nt = static_cast<size_t>(conv_tile_count(gr));
    NetLayout l{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += a256(b);
        return r;
    };
    l.dirs_f = take(n + 16);
    l.dirs_h = take(n + 16);
    l.feat = take(n * 32);
    l.a1 = take(n * 32);
    l.a2 = take(n * 32);
    l.p = take(n * 4);
    l.dz_a = take(n * 32);
    l.dz_b = take(n * 32);
    l.part = take(nt * 27 * 256 * 4);
    l.part_b = take(nt * 16 * 4);
    l.minmax = take(kConvBlocks * 2 * 4);
    l.L = take(n * 4);
    l.g0 = take(n * 4);
    l.total = o;
    return l;
}

struct Scratch2 {
    void* p = nullptr;
    hipStream_t s = nullptr;
    bool owned = false;
    ~Scratch2() {
        if (owned && p) (void)hipFreeAsync(p, s);
    }
    int get(void* user, size_t user_bytes, size_t need, hipStream_t stream) {
        s = stream;
        if (user) {
            if (user_bytes < need) return MSZ_EINVAL;
            p = user;
            return MSZ_OK;
        }
        if (hipMallocAsync(&p, need, stream) != hipSuccess) {
            p = nullptr;
            return MSZ_ENOMEM;
        }
        owned = true;
        return MSZ_OK;
    }
};

WeightView layer_view(const float* P, int layer) {
    switch (layer) {
        case 0: return {P + kOffW0, P + kOffB0, 256, 16, 1, 16, 16, 0};
        case 1: return {P + kOffW1, P + kOffB1, 256, 16, 1, 16, 16, 0};
        default: return {P + kOffW2, P + kOffB2, 16, 1, 0, 16, 1, 0};
    }
}

// Weights of the backward-data convolution of layer `layer` (transposed, taps flipped).
WeightView layer_back_view(const float* P, int layer) {
    if (layer == 1) return {P + kOffW1, nullptr, 256, 1, 16, 16, 16, 1};
    return {P + kOffW2, nullptr, 16, 0, 1, 1, 16, 1};  // layer 2: one input channel
}

void net_forward(const float* P, const uint16_t* feat, const Grid& gr, uint16_t* a1, uint16_t* a2, float* p,
                 hipStream_t s) {
    launch_conv_t<16, kConvHidden>(feat, gr, layer_view(P, 0), nullptr, a1, nullptr, s);
    launch_conv_t<16, kConvHidden>(a1, gr, layer_view(P, 1), nullptr, a2, nullptr, s);
    if (gr.nz == 1) {
        using T = ConvTile<32, 1>;
        const int nt = ((gr.nx + 15) / 16) * ((gr.ny + T::Y - 1) / T::Y);
        hipLaunchKernelGGL((k_conv_out<32, 1>), dim3(nt < kConvBlocks ? nt : kConvBlocks), dim3(256), 0, s, a2, gr,
                           P + kOffW2, P + kOffB2, p);
    } else {
        using T = ConvTile<8, 8>;
        const int nt = ((gr.nx + 15) / 16) * ((gr.ny + T::Y - 1) / T::Y) * ((gr.nz + T::Z - 1) / T::Z);
        hipLaunchKernelGGL((k_conv_out<8, 8>), dim3(nt < kConvBlocks ? nt : kConvBlocks), dim3(256), 0, s, a2, gr,
                           P + kOffW2, P + kOffB2, p);
    }
}

__global__ void __launch_bounds__(256) k_minmax(const float* __restrict__ f, int n, float* __restrict__ out) {
    __shared__ float smin[4], smax[4];
    float lo = INFINITY, hi = -INFINITY;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        lo = fminf(lo, f[i]);
        hi = fmaxf(hi, f[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
    }
    if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = lo, smax[threadIdx.x >> 6] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = fminf(fminf(smin[0], smin[1]), fminf(smin[2], smin[3]));
        out[2 * blockIdx.x + 1] = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    }
}

__global__ void __launch_bounds__(256) k_floor(const float* __restrict__ f, float xi, int n, float* __restrict__ L) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) L[i] = floor_bound(f[i], xi);
}

int blocks_n(long n) {
    long b = (n + 255) / 256;
    return static_cast<int>(b < 1 ? 1 : (b > kConvBlocks ? kConvBlocks : b));
}

int features_impl(const float* f, const float* fhat, const Grid& gr, float xi, uint16_t* feat, char* ws,
                  const NetLayout& l, hipStream_t s) {
    if (!(xi > 0.0f) || !(xi <= kValueLimit)) return MSZ_EINVAL;
    uint8_t* df = reinterpret_cast<uint8_t*>(ws + l.dirs_f);
    uint8_t* dh = reinterpret_cast<uint8_t*>(ws + l.dirs_h);
    float* mm = reinterpret_cast<float*>(ws + l.minmax);
    const int nb = blocks_n(gr.n);
    hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(256), 0, s, f, gr.n, mm);
    std::vector<float> host(2 * nb);
    if (hipMemcpyAsync(host.data(), mm, 2 * nb * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MSZ_EDEVICE;
    float lo = host[0], hi = host[1];
    for (int b = 1; b < nb; ++b) lo = fminf(lo, host[2 * b]), hi = fmaxf(hi, host[2 * b + 1]);
    const double range = static_cast<double>(hi) - static_cast<double>(lo);
    if (!(range > 0.0) || !std::isfinite(range)) return MSZ_EINVAL;
    const float xi_ch = static_cast<float>(std::log10(static_cast<double>(xi) / range) / 4.0 + 1.0);
    launch_dirs(f, gr, 0, df, s);
    launch_dirs(fhat, gr, 0, dh, s);
    hipLaunchKernelGGL(k_features, dim3(blocks_n(gr.nxy)), dim3(256), 0, s, f, fhat, df, dh, gr, xi, xi_ch, feat);
    return hipGetLastError() == hipSuccess ? MSZ_OK : MSZ_EDEVICE;
}

}  // namespace
}  // namespace msz

using namespace msz;

extern "C" {

size_t msz_net_workspace_bytes(msz_dims d) {
    Grid gr;
    if (!make_grid(d, gr)) return 0;
    return net_layout(gr).total;
}

size_t msz_learned_workspace_bytes(msz_dims d) {
    const size_t a = msz_net_workspace_bytes(d), b = msz_workspace_bytes(d);
    return a && b ? a256(a) + b : 0;
}

int msz_net_features(const float* f, const float* fhat, msz_dims d, float xi, uint16_t* feat, void* workspace,
                     size_t workspace_bytes, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !f || !fhat || !feat || !al16(feat)) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NetLayout l = net_layout(gr);
    Scratch2 ws;
    if (int rc = ws.get(workspace, workspace_bytes, l.total, s)) return rc;
    const int rc = features_impl(f, fhat, gr, xi, feat, static_cast<char*>(ws.p), l, s);
    if (rc) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? MSZ_OK : MSZ_EDEVICE;
}

int msz_net_halvings(const float* f, const float* fhat, const float* g, msz_dims d, float xi, float* k_out,
                     void* workspace, size_t workspace_bytes, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !f || !fhat || !g || !k_out) return MSZ_EINVAL;
    if (!(xi > 0.0f) || !(xi <= kValueLimit)) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Scratch2 ws;
    if (int rc = ws.get(workspace, workspace_bytes, a256(static_cast<size_t>(gr.n) * sizeof(float)), s)) return rc;
    float* L = static_cast<float*>(ws.p);
    hipLaunchKernelGGL(k_floor, dim3(blocks_n(gr.n)), dim3(256), 0, s, f, xi, gr.n, L);
    hipLaunchKernelGGL(k_halvings, dim3(blocks_n(gr.n)), dim3(256), 0, s, L, fhat, g, gr.n, k_out);
    if (hipGetLastError() != hipSuccess) return MSZ_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? MSZ_OK : MSZ_EDEVICE;
}

int msz_net_forward(const float* params, const uint16_t* feat, msz_dims d, float* p_out, uint16_t* act1_out,
                    uint16_t* act2_out, void* workspace, size_t workspace_bytes, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !params || !feat || !p_out || !al16(feat) || !al16(act1_out) || !al16(act2_out))
        return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NetLayout l = net_layout(gr);
    Scratch2 ws;
    if (int rc = ws.get(workspace, workspace_bytes, l.total, s)) return rc;
    char* w = static_cast<char*>(ws.p);
    uint16_t* a1 = act1_out ? act1_out : reinterpret_cast<uint16_t*>(w + l.a1);
    uint16_t* a2 = act2_out ? act2_out : reinterpret_cast<uint16_t*>(w + l.a2);
    net_forward(params, feat, gr, a1, a2, p_out, s);
    if (hipGetLastError() != hipSuccess) return MSZ_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? MSZ_OK : MSZ_EDEVICE;
}

int msz_net_gradients(const float* params, const uint16_t* feat, const float* target, float edit_weight, msz_dims d,
                      float* grad_out, float* loss_out, void* workspace, size_t workspace_bytes, void* stream) {
    Grid gr;
    if (!make_grid(d, gr) || !params || !feat || !target || !grad_out || !loss_out || !al16(feat)) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NetLayout l = net_layout(gr);
    Scratch2 ws;
    if (int rc = ws.get(workspace, workspace_bytes, l.total, s)) return rc;
    char* w = static_cast<char*>(ws.p);
    uint16_t* a1 = reinterpret_cast<uint16_t*>(w + l.a1);
    uint16_t* a2 = reinterpret_cast<uint16_t*>(w + l.a2);
    float* p = reinterpret_cast<float*>(w + l.p);
    uint16_t* dza = reinterpret_cast<uint16_t*>(w + l.dz_a);
    uint16_t* dzb = reinterpret_cast<uint16_t*>(w + l.dz_b);
    float* part = reinterpret_cast<float*>(w + l.part);
    float* part_b = reinterpret_cast<float*>(w + l.part_b);
    float* lp = reinterpret_cast<float*>(w + l.minmax);
    const int nt = conv_tile_count(gr);
    net_forward(params, feat, gr, a1, a2, p, s);
    const int nb = blocks_n(gr.n);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, p, target, gr.n, edit_weight, dza, lp);
    const int rb = (27 * 256 + 16 + 255) / 256;
    // layer 2
    launch_dw_t<16>(a2, dza, gr, part, part_b, s);
    hipLaunchKernelGGL(k_reduce_dw, dim3(rb), dim3(256), 0, s, part, part_b, nt, 16, 1, 1, grad_out + kOffW2,
                       grad_out + kOffB2);
    launch_conv_t<16, kConvBackData>(dza, gr, layer_back_view(params, 2), a2, dzb, nullptr, s);
    // layer 1
    launch_dw_t<16>(a1, dzb, gr, part, part_b, s);
    hipLaunchKernelGGL(k_reduce_dw, dim3(rb), dim3(256), 0, s, part, part_b, nt, 16, 16, 16, grad_out + kOffW1,
                       grad_out + kOffB1);
    launch_conv_t<16, kConvBackData>(dzb, gr, layer_back_view(params, 1), a1, dza, nullptr, s);
    // layer 0
    launch_dw_t<16>(feat, dza, gr, part, part_b, s);
    hipLaunchKernelGGL(k_reduce_dw, dim3(rb), dim3(256), 0, s, part, part_b, nt, 16, 16, 16, grad_out + kOffW0,
                       grad_out + kOffB0);
    if (hipGetLastError() != hipSuccess) return MSZ_EDEVICE;
    std::vector<float> host(nb);
    if (hipMemcpyAsync(host.data(), lp, nb * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MSZ_EDEVICE;
    double acc = 0.0;
    for (float v : host) acc += v;
    *loss_out = static_cast<float>(acc / gr.n);
    return MSZ_OK;
}

int msz_net_adam(float* params, const float* grad, float* m, float* v, int32_t n, int32_t step, float lr,
                 void* stream) {
    if (!params || !grad || !m || !v || n <= 0 || step < 1) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = static_cast<float>(1.0 - std::pow(0.9, step)), c2 = static_cast<float>(1.0 - std::pow(0.999, step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_n(n)), dim3(256), 0, s, params, grad, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
    if (hipGetLastError() != hipSuccess) return MSZ_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? MSZ_OK : MSZ_EDEVICE;
}

int msz_fix_learned(const float* f, const float* fhat, msz_dims d, float xi, const float* params, float p_min,
                    float* edits_out, const msz_options* opt, msz_stats* stats, void* stream) {
    if (!stats) return MSZ_EINVAL;
    std::memset(stats, 0, sizeof(*stats));
    Grid gr;
    msz_options o{};
    if (opt) o = *opt;
    if (!make_grid(d, gr) || !f || !fhat || !params || !edits_out || o.warm_start || !al16(f) || !al16(fhat)) {
        stats->status = MSZ_EINVAL;
        return MSZ_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NetLayout l = net_layout(gr);
    const size_t fix_bytes = msz_workspace_bytes(d);
    Scratch2 ws;
    if (int rc = ws.get(o.workspace, o.workspace_bytes, a256(l.total) + fix_bytes, s)) {
        stats->status = rc;
        return rc;
    }
    char* w = static_cast<char*>(ws.p);
    const bool timing = (o.flags & MSZ_FLAG_TIMING) != 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) return MSZ_EDEVICE;
    if (timing) (void)hipEventRecord(e0, s);
    uint16_t* feat = reinterpret_cast<uint16_t*>(w + l.feat);
    int rc = features_impl(f, fhat, gr, xi, feat, w, l, s);
    float* p = reinterpret_cast<float*>(w + l.p);
    float* L = reinterpret_cast<float*>(w + l.L);
    float* g0 = reinterpret_cast<float*>(w + l.g0);
    if (rc == MSZ_OK) {
        net_forward(params, feat, gr, reinterpret_cast<uint16_t*>(w + l.a1), reinterpret_cast<uint16_t*>(w + l.a2), p, s);
        hipLaunchKernelGGL(k_floor, dim3(blocks_n(gr.n)), dim3(256), 0, s, f, xi, gr.n, L);
        hipLaunchKernelGGL(k_warm_start, dim3(blocks_n(gr.n)), dim3(256), 0, s, p, L, fhat, p_min, gr.n, g0);
        if (hipGetLastError() != hipSuccess) rc = MSZ_EDEVICE;
    }
    if (timing) (void)hipEventRecord(e1, s);
    if (rc == MSZ_OK) {
        msz_options fo = o;
        fo.warm_start = g0;
        fo.workspace = w + a256(l.total);
        fo.workspace_bytes = fix_bytes;
        rc = msz_fix(f, fhat, d, xi, edits_out, &fo, stats, stream);
    } else {
        stats->status = rc;
    }
    if (timing) {
        float ms = 0.f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            stats->phase_ms[MSZ_PHASE_NET] = ms;
            stats->phase_launches[MSZ_PHASE_NET] = 1;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return rc;
}

}  // extern "C"
