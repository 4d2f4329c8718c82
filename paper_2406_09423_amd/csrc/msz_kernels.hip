// msz_kernels.hip -- gfx950 kernels of the MSz correction loop (arXiv 2406.09423).
//
// Data layout in HBM (one field of n vertices, x fastest):
//   h / g / L      float32[n]
//   dirs           uint8[n]   high nibble = ascent slot, low nibble = descent slot, 0xF = self
//   marks          uint8[n]   1 = "halve this vertex in the pending round" (padded to 16 B)
//   q_up, q_dn     int32[n]   pointer arrays of the ascending / descending forests
//   cnt            uint32[kSlots][kSlotStride] round counters, read back and summed by
//                  the host; block b adds into slot b % kSlots so that no cache line
//                  takes more than a few hundred atomics per launch
//
// Neighbour slots (Sec. 3 PL mesh; 2D uses slots 0..5, 3D all 14):
//   0 (+1,0,0)  1 (-1,0,0)  2 (0,+1,0)  3 (0,-1,0)  4 (+1,+1,0)  5 (-1,-1,0)
//   6 (0,0,+1)  7 (0,0,-1)  8 (+1,0,+1) 9 (-1,0,-1) 10 (0,+1,+1) 11 (0,-1,-1)
//   12 (+1,+1,+1) 13 (-1,-1,-1)
// The order (Sec. 4): a is above b iff h_a > h_b, or h_a == h_b and a > b.
#include "msz_internal.h"

namespace msz {

// ---------------------------------------------------------------- helpers ---

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide reduction of K counters followed by one atomic per non-zero total.
template <int K>
__device__ __forceinline__ void block_add(unsigned (&v)[K], unsigned* dst, const int* idx) {
    __shared__ unsigned red[K][16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        unsigned s = wave_sum(v[k]);
        if (lane == 0) red[k][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        unsigned s = 0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        if (s) atomicAdd(dst + (blockIdx.x & (kSlots - 1)) * kSlotStride + idx[threadIdx.x], s);
    }
}

// Proposals of one round form a set: every proposer of target t stores the
// same byte, so plain (idempotent) byte stores need no atomics.
__device__ __forceinline__ void mark(uint8_t* marks, int t) { marks[t] = 1; }

// One decreasing edit (Eqs. 2-6): halfway to the floor, snapped to it when
// float32 rounding would leave the value unchanged.
__device__ __forceinline__ float halve(float g, float L) {
    const float s = __fadd_rn(g, L);
    const float h = __fmul_rn(s, 0.5f);
    return h == g ? L : h;
}

__device__ __forceinline__ float f32_next_up(float x) {
    if (x == 0.0f) return __int_as_float(1);
    int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b + 1 : b - 1);
}

__device__ __forceinline__ float f32_next_down(float x) {
    if (x == 0.0f) return -__int_as_float(1);
    int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b - 1 : b + 1);
}

// Error-free difference a - b = s + e in binary64 (two-sum; no fused ops).
__device__ __forceinline__ void exact_diff(float a, float b, double& s, double& e) {
    const double da = a, nb = -static_cast<double>(b);
    s = __dadd_rn(da, nb);
    const double bv = __dadd_rn(s, -da);
    const double av = __dadd_rn(s, -bv);
    e = __dadd_rn(__dadd_rn(da, -av), __dadd_rn(nb, -bv));
}

// a - b <= c and a - b >= c, decided exactly.
__device__ __forceinline__ bool diff_at_most(float a, float b, float c) {
    double s, e;
    exact_diff(a, b, s, e);
    return s < static_cast<double>(c) || (s == static_cast<double>(c) && e <= 0.0);
}
__device__ __forceinline__ bool diff_at_least(float a, float b, float c) {
    double s, e;
    exact_diff(a, b, s, e);
    return s > static_cast<double>(c) || (s == static_cast<double>(c) && e >= 0.0);
}

// Smallest float32 L with L >= f - xi (the float reading of Eq. 1's bound).
__device__ __forceinline__ float floor_bound(float f, float xi) {
    float x = __double2float_rn(__dadd_rn(static_cast<double>(f), -static_cast<double>(xi)));
    for (int k = 0; k < 4 && !diff_at_most(f, x, xi); ++k) x = f32_next_up(x);
    for (int k = 0; k < 4; ++k) {
        const float y = f32_next_down(x);
        if (!diff_at_most(f, y, xi)) break;
        x = y;
    }
    return x;
}

__device__ __forceinline__ bool value_ok(float v) {
    return fabsf(v) <= kValueLimit;  // false for NaN and +-Inf
}

// ------------------------------------------------------ validate and init ---

// Checks the input contract, computes the floor L and the start field g.
// Four vertices per thread with dwordx4 accesses (arrays are 16-byte aligned);
// the last n % 4 vertices are handled one by one.
__device__ __forceinline__ void validate_one(float fi, float hi, const float* warm, int i, float xi,
                                             float& li, float& gi, unsigned& bad) {
    li = 0.0f;
    gi = hi;
    if (!value_ok(fi) || !value_ok(hi)) {
        bad |= kErrNonFinite;
        return;
    }
    if (!diff_at_most(fi, hi, xi) || !diff_at_least(fi, hi, -xi)) bad |= kErrBound;
    li = floor_bound(fi, xi);
    if (warm) {
        gi = warm[i];
        if (!value_ok(gi)) bad |= kErrWarmNonFinite;
        else if (!(gi >= li && gi <= hi)) bad |= kErrWarmBound;
    }
}

__global__ void __launch_bounds__(256) k_validate_init(const float* __restrict__ f,
                                                       const float* __restrict__ fhat,
                                                       const float* __restrict__ warm, float xi,
                                                       int n, float* __restrict__ L,
                                                       float* __restrict__ g,
                                                       unsigned* __restrict__ cnt) {
    unsigned bad = 0;
    const int ng = n >> 2;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < ng; w += gridDim.x * blockDim.x) {
        const float4 f4 = reinterpret_cast<const float4*>(f)[w];
        const float4 h4 = reinterpret_cast<const float4*>(fhat)[w];
        const float fv[4] = {f4.x, f4.y, f4.z, f4.w}, hv[4] = {h4.x, h4.y, h4.z, h4.w};
        float lv[4], gv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) validate_one(fv[j], hv[j], warm, 4 * w + j, xi, lv[j], gv[j], bad);
        reinterpret_cast<float4*>(L)[w] = make_float4(lv[0], lv[1], lv[2], lv[3]);
        reinterpret_cast<float4*>(g)[w] = make_float4(gv[0], gv[1], gv[2], gv[3]);
    }
    for (int i = 4 * ng + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float li, gi;
        validate_one(f[i], fhat[i], warm, i, xi, li, gi, bad);
        L[i] = li;
        g[i] = gi;
    }
    if (bad) atomicOr(cnt + kCntErr, bad);
}

// Finite-value check of a field handed to msz_labels / msz_count_false.
__global__ void __launch_bounds__(256) k_check_finite(const float* __restrict__ h, int n,
                                                      unsigned* __restrict__ cnt) {
    unsigned bad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (!value_ok(h[i])) bad = kErrNonFinite;
    if (bad) atomicOr(cnt + kCntErr, bad);
}

// ------------------------------------------------------------ detection ---

// The four C-loop predicates (Defs. 1-3) of vertex i from its packed
// directions in f (df) and g (dg); returns a bit per type and the edit
// target of type `type` (Eqs. 2-5; FPmin lowers dn_f, FNmax lowers up_g).
__device__ __forceinline__ unsigned c_cases(unsigned df, unsigned dg, int i, int type,
                                            const Grid& gr, int& target) {
    const unsigned uf = df >> 4, nf = df & 15u, ug = dg >> 4, ng = dg & 15u;
    const unsigned c0 = (ug == kSelf) & (uf != kSelf);   // FPmax
    const unsigned c1 = (ng == kSelf) & (nf != kSelf);   // FPmin
    const unsigned c2 = (uf == kSelf) & (ug != kSelf);   // FNmax
    const unsigned c3 = (nf == kSelf) & (ng != kSelf);   // FNmin
    switch (type) {
        case 0: target = i; break;
        case 1: target = i + gr.off[nf]; break;
        case 2: target = i + gr.off[ug]; break;
        default: target = i; break;
    }
    return c0 | (c1 << 1) | (c2 << 2) | (c3 << 3);
}

// Counts every C type and marks the targets of `type`.
__device__ __forceinline__ void detect_vertex(bool valid, unsigned df, unsigned dg, int i, int type,
                                              const Grid& gr, uint8_t* marks, unsigned (&c)[4]) {
    int t = 0;
    const unsigned bits = valid ? c_cases(df, dg, i, type, gr, t) : 0u;
    c[0] += bits & 1u;
    c[1] += (bits >> 1) & 1u;
    c[2] += (bits >> 2) & 1u;
    c[3] += (bits >> 3) & 1u;
    if ((bits >> type) & 1u) mark(marks, t);
}

// --------------------------------------------------- steepest directions ---
//
// Each block owns a 64 x TY tile of one z-slab of ZC planes.  Planes (with a
// one-vertex halo, NaN outside the grid so that it never wins a comparison)
// are staged in LDS and marched along z with a rolling window of three.  A
// thread computes four x-consecutive vertices of one row.
//
// MODE 0: write dirs only.  MODE 1: write dirs and run the C-loop detection
// of `type` against dirs_f.

struct TileCoord {
    int bx, by, bz;
};

// Maps the hardware block id to a tile so that consecutive tiles land on the
// same XCD (blocks are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, k = b & 7;
    return k * q + min(k, r) + (b >> 3);
}

template <int TY>
__device__ __forceinline__ void load_plane(float* __restrict__ dst, const float* __restrict__ h,
                                           const Grid& gr, int x0, int y0, int z) {
    constexpr int W = kTileX + 2, H = TY + 2;
    const bool zin = z >= 0 && z < gr.nz;
    const long base = static_cast<long>(z) * gr.nxy;
    for (int idx = threadIdx.x; idx < W * H; idx += blockDim.x) {
        const int r = idx / W, c = idx - r * W;
        const int x = x0 + c - 1, y = y0 + r - 1;
        float v = __builtin_nanf("");
        if (zin && x >= 0 && x < gr.nx && y >= 0 && y < gr.ny) v = h[base + x + static_cast<long>(gr.nx) * y];
        dst[idx] = v;
    }
}

struct Best {
    float uv, dv;
    int uo, dov;
    unsigned us, ds;
};

__device__ __forceinline__ void consider(Best& b, float w, int o, unsigned slot) {
    if (w > b.uv || (w == b.uv && o > b.uo)) {
        b.uv = w;
        b.uo = o;
        b.us = slot;
    }
    if (w < b.dv || (w == b.dv && o < b.dov)) {
        b.dv = w;
        b.dov = o;
        b.ds = slot;
    }
}

template <int NDIM, int TY, int ZC, int MODE>
__global__ void __launch_bounds__(16 * TY) k_dirs(const float* __restrict__ h, Grid gr,
                                                  uint8_t* __restrict__ dirs_out,
                                                  const uint8_t* __restrict__ dirs_f, int type,
                                                  uint8_t* __restrict__ marks,
                                                  unsigned* __restrict__ cnt) {
    constexpr int W = kTileX + 2, H = TY + 2, P = W * H;
    constexpr int NP = NDIM == 3 ? 3 : 1;
    __shared__ float sm[NP * P];

    const int tiles_x = (gr.nx + kTileX - 1) / kTileX;
    const int tiles_y = (gr.ny + TY - 1) / TY;
    const int nb = gridDim.x;
    const int lb = xcd_logical_block(blockIdx.x, nb);
    const int bx = lb % tiles_x;
    const int by = (lb / tiles_x) % tiles_y;
    const int bz = lb / (tiles_x * tiles_y);
    const int x0 = bx * kTileX, y0 = by * TY;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int y = y0 + ty;
    const int z0 = NDIM == 3 ? bz * ZC : 0;
    // rows start at multiples of 4 vertices: packed direction bytes move as dwords
    const bool vec4 = (gr.nx & 3) == 0;

    unsigned c[4] = {0u, 0u, 0u, 0u};

    int below = 0, cur = 0, above = 0;
    if constexpr (NDIM == 3) {
        load_plane<TY>(sm + 0 * P, h, gr, x0, y0, z0 - 1);
        load_plane<TY>(sm + 1 * P, h, gr, x0, y0, z0);
        below = 0;
        cur = 1;
        above = 2;
    } else {
        load_plane<TY>(sm, h, gr, x0, y0, 0);
    }

    const int zc = NDIM == 3 ? ZC : 1;
    for (int zz = 0; zz < zc; ++zz) {
        const int z = z0 + zz;
        if (z >= gr.nz) break;  // uniform across the block
        if constexpr (NDIM == 3) load_plane<TY>(sm + above * P, h, gr, x0, y0, z + 1);
        __syncthreads();
        const float* C = sm + cur * P;
        const float* A = sm + above * P;
        const float* B = sm + below * P;
        const int r = ty + 1;
        // the thread's four vertices: one dword of directions when rows are 4-aligned
        const int xa = x0 + tx * 4;
        const long i0 = static_cast<long>(z) * gr.nxy + static_cast<long>(gr.nx) * y + xa;
        const bool full = vec4 && xa + 3 < gr.nx && y < gr.ny;
        unsigned df4 = 0xFFFFFFFFu;
        if constexpr (MODE == 1) {
            if (full) {
                df4 = *reinterpret_cast<const unsigned*>(dirs_f + i0);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (xa + k < gr.nx && y < gr.ny)
                        df4 = (df4 & ~(0xFFu << (8 * k))) | (static_cast<unsigned>(dirs_f[i0 + k]) << (8 * k));
            }
        }
        unsigned out4 = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = xa + k;
            const int cc = tx * 4 + k + 1;
            const bool valid = x < gr.nx && y < gr.ny;
            const int i = static_cast<int>(i0) + k;
            unsigned packed = 0xFFu;
            if (valid) {
                const float v = C[r * W + cc];
                Best b{v, v, 0, 0, kSelf, kSelf};
                consider(b, C[r * W + cc + 1], gr.off[0], 0);
                consider(b, C[r * W + cc - 1], gr.off[1], 1);
                consider(b, C[(r + 1) * W + cc], gr.off[2], 2);
                consider(b, C[(r - 1) * W + cc], gr.off[3], 3);
                consider(b, C[(r + 1) * W + cc + 1], gr.off[4], 4);
                consider(b, C[(r - 1) * W + cc - 1], gr.off[5], 5);
                if constexpr (NDIM == 3) {
                    consider(b, A[r * W + cc], gr.off[6], 6);
                    consider(b, B[r * W + cc], gr.off[7], 7);
                    consider(b, A[r * W + cc + 1], gr.off[8], 8);
                    consider(b, B[r * W + cc - 1], gr.off[9], 9);
                    consider(b, A[(r + 1) * W + cc], gr.off[10], 10);
                    consider(b, B[(r - 1) * W + cc], gr.off[11], 11);
                    consider(b, A[(r + 1) * W + cc + 1], gr.off[12], 12);
                    consider(b, B[(r - 1) * W + cc - 1], gr.off[13], 13);
                }
                packed = (b.us << 4) | b.ds;
                out4 = (out4 & ~(0xFFu << (8 * k))) | (packed << (8 * k));
                if (!full) dirs_out[i0 + k] = static_cast<uint8_t>(packed);
            }
            if constexpr (MODE == 1) detect_vertex(valid, (df4 >> (8 * k)) & 0xFFu, packed, i, type, gr, marks, c);
        }
        if (full) *reinterpret_cast<unsigned*>(dirs_out + i0) = out4;
        __syncthreads();  // the oldest plane is overwritten next
        if constexpr (NDIM == 3) {
            const int t = below;
            below = cur;
            cur = above;
            above = t;
        }
    }
    if constexpr (MODE == 1) {
        const int idx[4] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3};
        block_add<4>(c, cnt, idx);
    }
}

// Detection from stored directions (g unchanged since they were computed).
// Four vertices per thread: one dword of each direction array.
__global__ void __launch_bounds__(256) k_detect_only(const uint8_t* __restrict__ dirs_f,
                                                     const uint8_t* __restrict__ dirs_g, Grid gr,
                                                     int type, uint8_t* __restrict__ marks,
                                                     unsigned* __restrict__ cnt) {
    unsigned c[4] = {0u, 0u, 0u, 0u};
    const int n = gr.n;
    const int ng = (n + 3) >> 2;
    // the direction arrays live in 256-byte padded workspace segments, so the
    // last partial dword can be read whole; lanes past n are masked
    const unsigned* wf = reinterpret_cast<const unsigned*>(dirs_f);
    const unsigned* wg = reinterpret_cast<const unsigned*>(dirs_g);
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < ng; w += gridDim.x * blockDim.x) {
        const unsigned df4 = wf[w], dg4 = wg[w];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * w + j;
            detect_vertex(i < n, (df4 >> (8 * j)) & 0xFFu, (dg4 >> (8 * j)) & 0xFFu, i, type, gr, marks, c);
        }
    }
    const int idx[4] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3};
    block_add<4>(c, cnt, idx);
}

// ---------------------------------------------------------------- apply ---

// Halves every marked vertex once (the round's union of proposals) and clears
// its mark.  Marks are scanned 16 at a time; the padding bytes are never set.
__global__ void __launch_bounds__(256) k_apply(float* __restrict__ g, const float* __restrict__ L,
                                               uint8_t* __restrict__ marks, int n,
                                               unsigned* __restrict__ cnt) {
    unsigned changed = 0;
    const int nw = (n + 15) >> 4;
    uint4* mw = reinterpret_cast<uint4*>(marks);
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
        const uint4 m = mw[w];
        if ((m.x | m.y | m.z | m.w) == 0u) continue;
        const unsigned part[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!part[q]) continue;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if ((part[q] >> (8 * b)) & 0xFFu) {
                    const int t = w * 16 + q * 4 + b;
                    const float old = g[t];
                    const float nv = halve(old, L[t]);
                    g[t] = nv;
                    changed += nv != old;
                }
            }
        }
        mw[w] = make_uint4(0u, 0u, 0u, 0u);
    }
    unsigned v[1] = {changed};
    const int idx[1] = {kCntChanged};
    block_add<1>(v, cnt, idx);
}

// --------------------------------------------------------------- labels ---
//
// Pointer jumping along the forests of steepest ascent and descent (Sec. 6.2).
// Stage 1 resolves each 4096-vertex tile inside LDS: every vertex ends up
// pointing at either the extremum it reaches inside its tile or the first
// vertex outside the tile on its integral line.  Such exit targets lie on the
// face layer of their own tile, so stage 2 only has to compress pointers of
// face-layer vertices (each thread walks its own chain, writing back every
// step; any value read is an ancestor, so no barrier is needed and each walk
// strictly advances).  Afterwards label(i) = q[q[i]].

template <int NDIM>
struct LabelTile;
template <>
struct LabelTile<2> {
    static constexpr int X = 64, Y = 64, Z = 1;
};
template <>
struct LabelTile<3> {
    static constexpr int X = 16, Y = 16, Z = 16;
};

__device__ __forceinline__ void slot_delta(unsigned s, int& dx, int& dy, int& dz) {
    // slots in the order of the table at the top of this file
    constexpr int DX[14] = {1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1};
    constexpr int DY[14] = {0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    constexpr int DZ[14] = {0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    dx = DX[s];
    dy = DY[s];
    dz = DZ[s];
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_label_tile(const uint8_t* __restrict__ dirs, Grid gr,
                                                    int* __restrict__ q_up,
                                                    int* __restrict__ q_dn) {
    using T = LabelTile<NDIM>;
    constexpr int NT = T::X * T::Y * T::Z;
    constexpr int PER = NT / 256;
    constexpr int PASSES = NDIM == 3 ? 12 : 12;  // 2^12 = 4096 >= any in-tile path
    __shared__ int su[NT];
    __shared__ int sd[NT];

    const int tx_n = (gr.nx + T::X - 1) / T::X;
    const int ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = lb % tx_n, by = (lb / tx_n) % ty_n, bz = lb / (tx_n * ty_n);
    const int X0 = bx * T::X, Y0 = by * T::Y, Z0 = bz * T::Z;

    // Thread t owns the 4-vertex row groups starting at l = 4 t + 1024 k.
    // Terminal pointers are stored as -(global id) - 1.
    const bool vec4 = (gr.nx & 3) == 0;
#pragma unroll
    for (int k = 0; k < PER / 4; ++k) {
        const int l0 = 4 * threadIdx.x + 1024 * k;
        const int lx0 = l0 % T::X, ly = (l0 / T::X) % T::Y, lz = l0 / (T::X * T::Y);
        const int xa = X0 + lx0, y = Y0 + ly, z = Z0 + lz;
        const bool row_in = y < gr.ny && z < gr.nz;
        const int i0 = xa + gr.nx * y + gr.nxy * z;
        unsigned d4 = 0xFFFFFFFFu;
        if (row_in && vec4 && xa + 3 < gr.nx) {
            d4 = *reinterpret_cast<const unsigned*>(dirs + i0);
        } else if (row_in) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (xa + j < gr.nx) d4 = (d4 & ~(0xFFu << (8 * j))) | (static_cast<unsigned>(dirs[i0 + j]) << (8 * j));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = l0 + j, lx = lx0 + j;
            int pu = -1, pd = -1;
            if (row_in && xa + j < gr.nx) {
                const int i = i0 + j;
                const unsigned d = (d4 >> (8 * j)) & 0xFFu;
                const unsigned s2[2] = {d >> 4, d & 15u};
                int p[2];
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const unsigned s = s2[w];
                    if (s == kSelf) {
                        p[w] = -i - 1;
                    } else {
                        int dx, dy, dz;
                        slot_delta(s, dx, dy, dz);
                        const int ax = lx + dx, ay = ly + dy, az = lz + dz;
                        if (ax >= 0 && ax < T::X && ay >= 0 && ay < T::Y && az >= 0 && az < T::Z)
                            p[w] = ax + T::X * (ay + T::Y * az);
                        else
                            p[w] = -(i + gr.off[s]) - 1;
                    }
                }
                pu = p[0];
                pd = p[1];
            }
            su[l] = pu;
            sd[l] = pd;
        }
    }
    __syncthreads();
    // doubling passes; stop early once every pointer of the tile is terminal
    for (int pass = 0; pass < PASSES; ++pass) {
        int pending = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int l = 4 * threadIdx.x + 1024 * (k >> 2) + (k & 3);
            const int a = su[l];
            if (a >= 0) {
                const int a2 = su[a];
                su[l] = a2;
                pending |= a2 >= 0;
            }
            const int b = sd[l];
            if (b >= 0) {
                const int b2 = sd[b];
                sd[l] = b2;
                pending |= b2 >= 0;
            }
        }
        if (!__syncthreads_or(pending)) break;
    }
    // Every in-tile path is shorter than the tile, so all pointers are terminal
    // here; a non-terminal one would still name an in-grid ancestor.
    auto global_of = [&](int a) {
        return a < 0 ? -a - 1
                     : X0 + a % T::X + gr.nx * (Y0 + (a / T::X) % T::Y) + gr.nxy * (Z0 + a / (T::X * T::Y));
    };
#pragma unroll
    for (int k = 0; k < PER / 4; ++k) {
        const int l0 = 4 * threadIdx.x + 1024 * k;
        const int lx0 = l0 % T::X, ly = (l0 / T::X) % T::Y, lz = l0 / (T::X * T::Y);
        const int xa = X0 + lx0, y = Y0 + ly, z = Z0 + lz;
        if (y >= gr.ny || z >= gr.nz) continue;
        const int i0 = xa + gr.nx * y + gr.nxy * z;
        if (vec4 && xa + 3 < gr.nx) {
            *reinterpret_cast<int4*>(q_up + i0) =
                make_int4(global_of(su[l0]), global_of(su[l0 + 1]), global_of(su[l0 + 2]), global_of(su[l0 + 3]));
            *reinterpret_cast<int4*>(q_dn + i0) =
                make_int4(global_of(sd[l0]), global_of(sd[l0 + 1]), global_of(sd[l0 + 2]), global_of(sd[l0 + 3]));
        } else {
            for (int j = 0; j < 4 && xa + j < gr.nx; ++j) {
                q_up[i0 + j] = global_of(su[l0 + j]);
                q_dn[i0 + j] = global_of(sd[l0 + j]);
            }
        }
    }
}

// Number of face-layer vertices of a full label tile.
template <int NDIM>
__host__ __device__ constexpr int face_count() {
    using T = LabelTile<NDIM>;
    return NDIM == 2 ? 2 * T::X + 2 * (T::Y - 2)
                     : 2 * T::X * T::Y + 2 * T::X * (T::Z - 2) + 2 * (T::Y - 2) * (T::Z - 2);
}

// b-th face-layer vertex of a tile, in local coordinates.
template <int NDIM>
__device__ __forceinline__ void face_vertex(int b, int& lx, int& ly, int& lz) {
    using T = LabelTile<NDIM>;
    if constexpr (NDIM == 2) {
        lz = 0;
        if (b < 2 * T::X) {
            lx = b % T::X;
            ly = (b / T::X) ? T::Y - 1 : 0;
        } else {
            b -= 2 * T::X;
            ly = 1 + b % (T::Y - 2);
            lx = (b / (T::Y - 2)) ? T::X - 1 : 0;
        }
    } else {
        const int A = T::X * T::Y;
        if (b < 2 * A) {  // z faces
            lx = b % T::X;
            ly = (b / T::X) % T::Y;
            lz = (b / A) ? T::Z - 1 : 0;
            return;
        }
        b -= 2 * A;
        const int Bn = T::X * (T::Z - 2);
        if (b < 2 * Bn) {  // y faces
            lx = b % T::X;
            lz = 1 + (b / T::X) % (T::Z - 2);
            ly = (b / Bn) ? T::Y - 1 : 0;
            return;
        }
        b -= 2 * Bn;
        const int Cn = (T::Y - 2) * (T::Z - 2);  // x faces
        ly = 1 + b % (T::Y - 2);
        lz = 1 + (b / (T::Y - 2)) % (T::Z - 2);
        lx = (b / Cn) ? T::X - 1 : 0;
    }
}

__device__ __forceinline__ int load_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Walks q[x] to the root of x's forest, writing every step back.  The forests
// are acyclic (every pointer goes strictly up, resp. down, the total order), so
// the walk ends; the step cap only guards against corrupted input and is
// reported as an error.
constexpr int kMaxWalk = 1 << 22;
__device__ __forceinline__ bool compress_one(int* q, int x) {
    int y = load_relaxed(q + x);
    for (int it = 0; it < kMaxWalk; ++it) {
        const int z = load_relaxed(q + y);
        if (z == y) return true;  // only roots point at themselves
        store_relaxed(q + x, z);
        y = z;
    }
    return false;
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_label_compress(Grid gr, int* __restrict__ q_up,
                                                        int* __restrict__ q_dn,
                                                        unsigned* __restrict__ cnt) {
    using T = LabelTile<NDIM>;
    constexpr int FC = face_count<NDIM>();
    const int tx_n = (gr.nx + T::X - 1) / T::X;
    const int ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = lb % tx_n, by = (lb / tx_n) % ty_n, bz = lb / (tx_n * ty_n);
    for (int b = threadIdx.x; b < FC; b += blockDim.x) {
        int lx, ly, lz;
        face_vertex<NDIM>(b, lx, ly, lz);
        const int x = bx * T::X + lx, y = by * T::Y + ly, z = bz * T::Z + lz;
        if (x >= gr.nx || y >= gr.ny || z >= gr.nz) continue;
        const int i = x + gr.nx * y + gr.nxy * z;
        const bool ok_up = compress_one(q_up, i);
        const bool ok_dn = compress_one(q_dn, i);
        const bool ok = ok_up && ok_dn;
        if (!ok) atomicOr(cnt + kCntErr, kErrWalk);
    }
}

// Writes the final labels label(i) = q[q[i]].  May run in place (M == q_up,
// m == q_dn): the values it reads are fixed points.  Arrays are 16-byte aligned.
__global__ void __launch_bounds__(256) k_label_final(const int* q_up, const int* q_dn, int n, int* M,
                                                     int* m) {
    const int ng = n >> 2;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < ng; w += gridDim.x * blockDim.x) {
        const int4 a = reinterpret_cast<const int4*>(q_up)[w];
        const int4 b = reinterpret_cast<const int4*>(q_dn)[w];
        const int4 ra = make_int4(q_up[a.x], q_up[a.y], q_up[a.z], q_up[a.w]);
        const int4 rb = make_int4(q_dn[b.x], q_dn[b.y], q_dn[b.z], q_dn[b.w]);
        reinterpret_cast<int4*>(M)[w] = ra;
        reinterpret_cast<int4*>(m)[w] = rb;
    }
    for (int i = 4 * ng + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        M[i] = q_up[q_up[i]];
        m[i] = q_dn[q_dn[i]];
    }
}

// ------------------------------------------------------- R-loop detection ---
//
// Four vertices per thread (dword / dwordx4 accesses of the padded workspace arrays).
__global__ void __launch_bounds__(256) k_detect_r(const uint8_t* __restrict__ dirs_f,
                                                  const uint8_t* __restrict__ dirs_g,
                                                  const int* __restrict__ q_up,
                                                  const int* __restrict__ q_dn,
                                                  const int* __restrict__ Mf,
                                                  const int* __restrict__ mf, Grid gr,
                                                  uint8_t* __restrict__ marks,
                                                  unsigned* __restrict__ cnt) {
    unsigned wrong = 0, cases = 0;
    const int n = gr.n;
    const int ng = (n + 3) >> 2;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < ng; w += gridDim.x * blockDim.x) {
        const unsigned df4 = reinterpret_cast<const unsigned*>(dirs_f)[w];
        const unsigned dg4 = reinterpret_cast<const unsigned*>(dirs_g)[w];
        const int4 qu4 = reinterpret_cast<const int4*>(q_up)[w];
        const int4 qd4 = reinterpret_cast<const int4*>(q_dn)[w];
        const int4 Mf4 = reinterpret_cast<const int4*>(Mf)[w];
        const int4 mf4 = reinterpret_cast<const int4*>(mf)[w];
        const int qu[4] = {qu4.x, qu4.y, qu4.z, qu4.w}, qd[4] = {qd4.x, qd4.y, qd4.z, qd4.w};
        const int Mv[4] = {Mf4.x, Mf4.y, Mf4.z, Mf4.w}, mv[4] = {mf4.x, mf4.y, mf4.z, mf4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * w + j;
            if (i >= n) break;
            const unsigned df = (df4 >> (8 * j)) & 0xFFu, dg = (dg4 >> (8 * j)) & 0xFFu;
            const bool wM = q_up[qu[j]] != Mv[j];
            const bool wm = q_dn[qd[j]] != mv[j];
            wrong += wM || wm;
            const bool rmin = wm && ((dg & 15u) != (df & 15u));
            const bool rmax = wM && ((dg >> 4) != (df >> 4));
            cases += rmin + rmax;
            if (rmin) mark(marks, i + gr.off[df & 15u]);
            if (rmax) mark(marks, i + gr.off[dg >> 4]);
        }
    }
    unsigned v[2] = {wrong, cases};
    const int idx[2] = {kCntWrong, kCntRCases};
    block_add<2>(v, cnt, idx);
}

// ------------------------------------------------ count_false comparison ---
__global__ void __launch_bounds__(256) k_compare(const uint8_t* __restrict__ dirs_f,
                                                 const uint8_t* __restrict__ dirs_g,
                                                 const int* __restrict__ qfu,
                                                 const int* __restrict__ qfd,
                                                 const int* __restrict__ qgu,
                                                 const int* __restrict__ qgd, int n,
                                                 unsigned* __restrict__ cnt) {
    unsigned c[7] = {0, 0, 0, 0, 0, 0, 0};
    Grid dummy{};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int t;
        const unsigned bits = c_cases(dirs_f[i], dirs_g[i], i, 0, dummy, t);
        c[0] += bits & 1u;
        c[1] += (bits >> 1) & 1u;
        c[2] += (bits >> 2) & 1u;
        c[3] += (bits >> 3) & 1u;
        const bool wM = qgu[qgu[i]] != qfu[qfu[i]];
        const bool wm = qgd[qgd[i]] != qfd[qfd[i]];
        c[4] += wM;
        c[5] += wm;
        c[6] += wM || wm;
    }
    const int idx[7] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3,
                        kCntWrongMax, kCntWrongMin, kCntWrong};
    block_add<7>(c, cnt, idx);
}

// ---------------------------------------------------------------- output ---
//
// delta = fl(g - fhat); when fl(fhat + delta) misses g, the floats up to two
// ulps either side are tried in the order +1, -1, +2, -2.
__device__ __forceinline__ float delta_one(float gi, float hi, unsigned& edited, unsigned& inexact) {
    const float d0 = __fsub_rn(gi, hi);
    float d = d0;
    bool ok = __fadd_rn(hi, d0) == gi;
    if (!ok) {
        const float up1 = f32_next_up(d0), dn1 = f32_next_down(d0);
        const float cand[4] = {up1, dn1, f32_next_up(up1), f32_next_down(dn1)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok && __fadd_rn(hi, cand[k]) == gi) {
                d = cand[k];
                ok = true;
            }
        }
    }
    edited += gi != hi;
    inexact += !ok;
    return ok ? d : d0;
}

__global__ void __launch_bounds__(256) k_delta(const float* __restrict__ g,
                                               const float* __restrict__ fhat, int n,
                                               float* __restrict__ delta,
                                               float* __restrict__ g_out,
                                               unsigned* __restrict__ cnt) {
    unsigned edited = 0, inexact = 0;
    const int ng = n >> 2;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < ng; w += gridDim.x * blockDim.x) {
        const float4 g4 = reinterpret_cast<const float4*>(g)[w];
        const float4 h4 = reinterpret_cast<const float4*>(fhat)[w];
        const float4 d4 = make_float4(delta_one(g4.x, h4.x, edited, inexact),
                                      delta_one(g4.y, h4.y, edited, inexact),
                                      delta_one(g4.z, h4.z, edited, inexact),
                                      delta_one(g4.w, h4.w, edited, inexact));
        reinterpret_cast<float4*>(delta)[w] = d4;
        if (g_out) reinterpret_cast<float4*>(g_out)[w] = g4;
    }
    for (int i = 4 * ng + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        delta[i] = delta_one(gi, fhat[i], edited, inexact);
        if (g_out) g_out[i] = gi;
    }
    unsigned v[2] = {edited, inexact};
    const int idx[2] = {kCntEdited, kCntInexact};
    block_add<2>(v, cnt, idx);
}

// ================================================================ launchers ==

static int blocks_for(long work, int per_block, int cap = 1 << 20) {
    long b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<int>(b);
}

struct DirsVariant {
    int ty, zc;
};
// Tile variants selectable per launch (index 1..); index 0 is the default.
static const DirsVariant kVariants2D[] = {{16, 1}, {16, 1}, {8, 1}, {4, 1}};
static const DirsVariant kVariants3D[] = {{8, 16}, {16, 16}, {8, 16}, {4, 32}, {16, 8}, {8, 8}};

int tile_variant_count(int ndim) {
    return ndim == 2 ? static_cast<int>(sizeof(kVariants2D) / sizeof(kVariants2D[0])) - 1
                     : static_cast<int>(sizeof(kVariants3D) / sizeof(kVariants3D[0])) - 1;
}

template <int NDIM, int TY, int ZC, int MODE>
static void launch_dirs_t(const float* h, const Grid& gr, uint8_t* dirs_out, const uint8_t* dirs_f,
                          int type, uint8_t* marks, unsigned* cnt, hipStream_t s) {
    const int tx = (gr.nx + kTileX - 1) / kTileX;
    const int ty = (gr.ny + TY - 1) / TY;
    const int tz = NDIM == 3 ? (gr.nz + ZC - 1) / ZC : 1;
    const int nb = tx * ty * tz;
    hipLaunchKernelGGL((k_dirs<NDIM, TY, ZC, MODE>), dim3(nb), dim3(16 * TY), 0, s, h, gr, dirs_out,
                       dirs_f, type, marks, cnt);
}

template <int MODE>
static void launch_dirs_mode(const float* h, const Grid& gr, int variant, uint8_t* dirs_out,
                             const uint8_t* dirs_f, int type, uint8_t* marks,
                             unsigned* cnt, hipStream_t s) {
    if (gr.ndim == 2) {
        const int ty = kVariants2D[variant].ty;
        if (ty == 16) launch_dirs_t<2, 16, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else if (ty == 8) launch_dirs_t<2, 8, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else launch_dirs_t<2, 4, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
    } else {
        const DirsVariant v = kVariants3D[variant];
        if (v.ty == 16 && v.zc == 16) launch_dirs_t<3, 16, 16, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else if (v.ty == 8 && v.zc == 16) launch_dirs_t<3, 8, 16, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else if (v.ty == 4 && v.zc == 32) launch_dirs_t<3, 4, 32, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else if (v.ty == 16 && v.zc == 8) launch_dirs_t<3, 16, 8, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
        else launch_dirs_t<3, 8, 8, MODE>(h, gr, dirs_out, dirs_f, type, marks, cnt, s);
    }
}

void launch_dirs(const float* h, const Grid& gr, int variant, uint8_t* dirs_out, hipStream_t s) {
    launch_dirs_mode<0>(h, gr, variant, dirs_out, nullptr, 0, nullptr, nullptr, s);
}

void launch_dirs_detect(const float* g, const Grid& gr, int variant, uint8_t* dirs_g,
                        const uint8_t* dirs_f, int type, uint8_t* marks, unsigned* cnt,
                        hipStream_t s) {
    launch_dirs_mode<1>(g, gr, variant, dirs_g, dirs_f, type, marks, cnt, s);
}

void launch_detect_only(const uint8_t* dirs_f, const uint8_t* dirs_g, const Grid& gr, int type,
                        uint8_t* marks, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_detect_only, dim3(blocks_for((gr.n + 3) / 4, 256, kGridCap)), dim3(256), 0, s, dirs_f,
                       dirs_g, gr, type, marks, cnt);
}

void launch_apply(float* g, const float* L, uint8_t* marks, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_apply, dim3(blocks_for((n + 15) / 16, 256, kGridCap)), dim3(256), 0, s, g, L,
                       marks, n, cnt);
}

static int label_tiles(const Grid& gr) {
    if (gr.ndim == 2) {
        using T = LabelTile<2>;
        return ((gr.nx + T::X - 1) / T::X) * ((gr.ny + T::Y - 1) / T::Y);
    }
    using T = LabelTile<3>;
    return ((gr.nx + T::X - 1) / T::X) * ((gr.ny + T::Y - 1) / T::Y) * ((gr.nz + T::Z - 1) / T::Z);
}

void launch_label_tile(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, hipStream_t s) {
    const int nb = label_tiles(gr);
    if (gr.ndim == 2) hipLaunchKernelGGL(k_label_tile<2>, dim3(nb), dim3(256), 0, s, dirs, gr, q_up, q_dn);
    else hipLaunchKernelGGL(k_label_tile<3>, dim3(nb), dim3(256), 0, s, dirs, gr, q_up, q_dn);
}

void launch_label_compress(const Grid& gr, int* q_up, int* q_dn, unsigned* cnt, hipStream_t s) {
    const int nb = label_tiles(gr);
    if (gr.ndim == 2) hipLaunchKernelGGL(k_label_compress<2>, dim3(nb), dim3(256), 0, s, gr, q_up, q_dn, cnt);
    else hipLaunchKernelGGL(k_label_compress<3>, dim3(nb), dim3(256), 0, s, gr, q_up, q_dn, cnt);
}

void launch_label_forests(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, unsigned* cnt,
                          hipStream_t s) {
    launch_label_tile(dirs, gr, q_up, q_dn, s);
    launch_label_compress(gr, q_up, q_dn, cnt, s);
}

void launch_label_final(const int* q_up, const int* q_dn, int n, int* M, int* m, hipStream_t s) {
    hipLaunchKernelGGL(k_label_final, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, q_up, q_dn,
                       n, M, m);
}

void launch_detect_r(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* q_up, const int* q_dn,
                     const int* Mf, const int* mf, const Grid& gr, uint8_t* marks,
                     unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_detect_r, dim3(blocks_for((gr.n + 3) / 4, 256, kGridCap)), dim3(256), 0, s, dirs_f,
                       dirs_g, q_up, q_dn, Mf, mf, gr, marks, cnt);
}

void launch_compare(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* qfu, const int* qfd,
                    const int* qgu, const int* qgd, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_compare, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, dirs_f, dirs_g,
                       qfu, qfd, qgu, qgd, n, cnt);
}

void launch_validate_init(const float* f, const float* fhat, const float* warm, float xi, int n,
                          float* L, float* g, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_validate_init, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, f, fhat,
                       warm, xi, n, L, g, cnt);
}

void launch_check_finite(const float* h, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, h, n, cnt);
}

void launch_delta(const float* g, const float* fhat, int n, float* delta, float* g_out, unsigned* cnt,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_delta, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, g, fhat, n, delta,
                       g_out, cnt);
}

}  // namespace msz
