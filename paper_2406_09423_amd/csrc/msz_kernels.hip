// msz_kernels.hip -- gfx950 kernels of the MSz correction loop (arXiv 2406.09423).
//
// Data layout in HBM (one field of n vertices, x fastest):
//   h / g / L      float32[n]
//   dirs           uint8[n]   high nibble = ascent slot, low nibble = descent slot, 0xF = self
//   marks          uint8[n]   1 = "halve this vertex in the pending round" (padded to 4 B)
//   q_up, q_dn     int32[n]   pointer arrays of the ascending / descending forests
//   list           int32[n]   compacted, duplicate-free edit targets of one round
//   cnt            uint32[64] round counters read back by the host
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
        if (s) atomicAdd(dst + idx[threadIdx.x], s);
    }
}

// Claims vertex t for the pending round; true for exactly one caller per round.
__device__ __forceinline__ bool claim_mark(uint8_t* marks, int t) {
    unsigned* w = reinterpret_cast<unsigned*>(marks + (t & ~3));
    const unsigned bit = 1u << ((t & 3) * 8);
    return (atomicOr(w, bit) & bit) == 0;
}

// Appends the claimed targets of a wave to the round's list with one atomic per wave.
__device__ __forceinline__ void push_targets(bool claimed, int t, int* list, unsigned* len) {
    const unsigned long long m = __ballot(claimed);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll(static_cast<long long>(m)) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(len, static_cast<unsigned>(__popcll(m)));
    base = __shfl(base, leader);
    if (claimed) {
        const unsigned rank = __popcll(m & ((1ull << lane) - 1ull));
        list[base + rank] = t;
    }
}

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
__global__ void __launch_bounds__(256) k_validate_init(const float* __restrict__ f,
                                                       const float* __restrict__ fhat,
                                                       const float* __restrict__ warm, float xi,
                                                       int n, float* __restrict__ L,
                                                       float* __restrict__ g,
                                                       unsigned* __restrict__ cnt) {
    unsigned bad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float fi = f[i], hi = fhat[i];
        if (!value_ok(fi) || !value_ok(hi)) {
            bad |= kErrNonFinite;
            continue;
        }
        if (!diff_at_most(fi, hi, xi) || !diff_at_least(fi, hi, -xi)) bad |= kErrBound;
        const float li = floor_bound(fi, xi);
        L[i] = li;
        float gi = hi;
        if (warm) {
            gi = warm[i];
            if (!value_ok(gi)) bad |= kErrWarmNonFinite;
            else if (!(gi >= li && gi <= hi)) bad |= kErrWarmBound;
        }
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

// Counts every C type, marks and lists the targets of `type`.
__device__ __forceinline__ void detect_vertex(bool valid, unsigned df, unsigned dg, int i, int type,
                                              const Grid& gr, uint8_t* marks, int* list,
                                              unsigned* cnt, unsigned (&c)[4]) {
    int t = 0;
    const unsigned bits = valid ? c_cases(df, dg, i, type, gr, t) : 0u;
    c[0] += bits & 1u;
    c[1] += (bits >> 1) & 1u;
    c[2] += (bits >> 2) & 1u;
    c[3] += (bits >> 3) & 1u;
    const bool hit = (bits >> type) & 1u;
    const bool claimed = hit && claim_mark(marks, t);
    push_targets(claimed, t, list, cnt + kCntList);
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
                                                  uint8_t* __restrict__ marks, int* __restrict__ list,
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
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + tx * 4 + k;
            const int cc = tx * 4 + k + 1;
            const bool valid = x < gr.nx && y < gr.ny;
            const long ii = static_cast<long>(z) * gr.nxy + static_cast<long>(gr.nx) * y + x;
            const int i = static_cast<int>(ii);
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
                dirs_out[ii] = static_cast<uint8_t>(packed);
            }
            if constexpr (MODE == 1) {
                const unsigned df = valid ? dirs_f[ii] : 0xFFu;
                detect_vertex(valid, df, packed, i, type, gr, marks, list, cnt, c);
            }
        }
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
__global__ void __launch_bounds__(256) k_detect_only(const uint8_t* __restrict__ dirs_f,
                                                     const uint8_t* __restrict__ dirs_g, Grid gr,
                                                     int type, uint8_t* __restrict__ marks,
                                                     int* __restrict__ list,
                                                     unsigned* __restrict__ cnt) {
    unsigned c[4] = {0u, 0u, 0u, 0u};
    const int n = gr.n;
    const int stride = gridDim.x * blockDim.x;
    // loop bound is uniform across each wave so the ballots stay convergent
    const int iters = (n + stride - 1) / stride;
    for (int it = 0; it < iters; ++it) {
        const int i = it * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = i < n;
        const unsigned df = valid ? dirs_f[i] : 0xFFu;
        const unsigned dg = valid ? dirs_g[i] : 0xFFu;
        detect_vertex(valid, df, dg, i, type, gr, marks, list, cnt, c);
    }
    const int idx[4] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3};
    block_add<4>(c, cnt, idx);
}

// ---------------------------------------------------------------- apply ---

// Halves every listed target once (the round's union of proposals) and clears its mark.
__global__ void __launch_bounds__(256) k_apply(const int* __restrict__ list, int len,
                                               float* __restrict__ g, const float* __restrict__ L,
                                               uint8_t* __restrict__ marks,
                                               unsigned* __restrict__ cnt) {
    unsigned changed = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < len; k += gridDim.x * blockDim.x) {
        const int t = list[k];
        const float old = g[t];
        const float nv = halve(old, L[t]);
        g[t] = nv;
        marks[t] = 0;
        changed += nv != old;
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

    // terminal pointers are stored as -(global id) - 1
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int l = threadIdx.x + k * 256;
        const int lx = l % T::X, ly = (l / T::X) % T::Y, lz = l / (T::X * T::Y);
        const int x = X0 + lx, y = Y0 + ly, z = Z0 + lz;
        int pu = -1, pd = -1;
        if (x < gr.nx && y < gr.ny && z < gr.nz) {
            const int i = x + gr.nx * y + gr.nxy * z;
            const unsigned d = dirs[i];
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
    __syncthreads();
    for (int pass = 0; pass < PASSES; ++pass) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int l = threadIdx.x + k * 256;
            const int a = su[l];
            if (a >= 0) su[l] = su[a];
            const int b = sd[l];
            if (b >= 0) sd[l] = sd[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int l = threadIdx.x + k * 256;
        const int lx = l % T::X, ly = (l / T::X) % T::Y, lz = l / (T::X * T::Y);
        const int x = X0 + lx, y = Y0 + ly, z = Z0 + lz;
        if (x < gr.nx && y < gr.ny && z < gr.nz) {
            const int i = x + gr.nx * y + gr.nxy * z;
            // every in-tile path is shorter than the tile, so all pointers are terminal
            // here; a non-terminal one would still name an in-grid ancestor
            const int a = su[l], b = sd[l];
            q_up[i] = a < 0 ? -a - 1 : X0 + a % T::X + gr.nx * (Y0 + (a / T::X) % T::Y) + gr.nxy * (Z0 + a / (T::X * T::Y));
            q_dn[i] = b < 0 ? -b - 1 : X0 + b % T::X + gr.nx * (Y0 + (b / T::X) % T::Y) + gr.nxy * (Z0 + b / (T::X * T::Y));
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

// Writes the final labels label(i) = q[q[i]].
// May run in place (M == q_up, m == q_dn): the values it reads are fixed points.
__global__ void __launch_bounds__(256) k_label_final(const int* q_up, const int* q_dn, int n, int* M,
                                                     int* m) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        M[i] = q_up[q_up[i]];
        m[i] = q_dn[q_dn[i]];
    }
}

// ------------------------------------------------------- R-loop detection ---
//
// A vertex u is a troublemaker when its steepest step in g leaves the one in
// f while its label is wrong (Sec. 5.2); the first divergence on the integral
// line of any mislabelled vertex is such a vertex, and every such vertex is
// its own first divergence.  Wrong minimum: lower dn_f(u); wrong maximum:
// lower up_g(u) (Eq. 6 under value-lowering edits).
__global__ void __launch_bounds__(256) k_detect_r(const uint8_t* __restrict__ dirs_f,
                                                  const uint8_t* __restrict__ dirs_g,
                                                  const int* __restrict__ q_up,
                                                  const int* __restrict__ q_dn,
                                                  const int* __restrict__ Mf,
                                                  const int* __restrict__ mf, Grid gr,
                                                  uint8_t* __restrict__ marks,
                                                  int* __restrict__ list,
                                                  unsigned* __restrict__ cnt) {
    unsigned wrong = 0, cases = 0;
    const int n = gr.n;
    const int stride = gridDim.x * blockDim.x;
    const int iters = (n + stride - 1) / stride;
    for (int it = 0; it < iters; ++it) {
        const int i = it * stride + blockIdx.x * blockDim.x + threadIdx.x;
        bool rmin = false, rmax = false;
        int tmin = 0, tmax = 0;
        if (i < n) {
            const unsigned df = dirs_f[i], dg = dirs_g[i];
            const bool wM = q_up[q_up[i]] != Mf[i];
            const bool wm = q_dn[q_dn[i]] != mf[i];
            wrong += wM || wm;
            rmin = wm && ((dg & 15u) != (df & 15u));
            rmax = wM && ((dg >> 4) != (df >> 4));
            tmin = i + gr.off[df & 15u];
            tmax = i + gr.off[dg >> 4];
            cases += rmin + rmax;
        }
        const bool c1 = rmin && claim_mark(marks, tmin);
        push_targets(c1, tmin, list, cnt + kCntList);
        const bool c2 = rmax && claim_mark(marks, tmax);
        push_targets(c2, tmax, list, cnt + kCntList);
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
__global__ void __launch_bounds__(256) k_delta(const float* __restrict__ g,
                                               const float* __restrict__ fhat, int n,
                                               float* __restrict__ delta,
                                               float* __restrict__ g_out,
                                               unsigned* __restrict__ cnt) {
    unsigned edited = 0, inexact = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i], hi = fhat[i];
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
        delta[i] = ok ? d : d0;
        if (g_out) g_out[i] = gi;
        edited += gi != hi;
        inexact += !ok;
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
                          int type, uint8_t* marks, int* list, unsigned* cnt, hipStream_t s) {
    const int tx = (gr.nx + kTileX - 1) / kTileX;
    const int ty = (gr.ny + TY - 1) / TY;
    const int tz = NDIM == 3 ? (gr.nz + ZC - 1) / ZC : 1;
    const int nb = tx * ty * tz;
    hipLaunchKernelGGL((k_dirs<NDIM, TY, ZC, MODE>), dim3(nb), dim3(16 * TY), 0, s, h, gr, dirs_out,
                       dirs_f, type, marks, list, cnt);
}

template <int MODE>
static void launch_dirs_mode(const float* h, const Grid& gr, int variant, uint8_t* dirs_out,
                             const uint8_t* dirs_f, int type, uint8_t* marks, int* list,
                             unsigned* cnt, hipStream_t s) {
    if (gr.ndim == 2) {
        const int ty = kVariants2D[variant].ty;
        if (ty == 16) launch_dirs_t<2, 16, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else if (ty == 8) launch_dirs_t<2, 8, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else launch_dirs_t<2, 4, 1, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
    } else {
        const DirsVariant v = kVariants3D[variant];
        if (v.ty == 16 && v.zc == 16) launch_dirs_t<3, 16, 16, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else if (v.ty == 8 && v.zc == 16) launch_dirs_t<3, 8, 16, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else if (v.ty == 4 && v.zc == 32) launch_dirs_t<3, 4, 32, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else if (v.ty == 16 && v.zc == 8) launch_dirs_t<3, 16, 8, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
        else launch_dirs_t<3, 8, 8, MODE>(h, gr, dirs_out, dirs_f, type, marks, list, cnt, s);
    }
}

void launch_dirs(const float* h, const Grid& gr, int variant, uint8_t* dirs_out, hipStream_t s) {
    launch_dirs_mode<0>(h, gr, variant, dirs_out, nullptr, 0, nullptr, nullptr, nullptr, s);
}

void launch_dirs_detect(const float* g, const Grid& gr, int variant, uint8_t* dirs_g,
                        const uint8_t* dirs_f, int type, uint8_t* marks, int* list, unsigned* cnt,
                        hipStream_t s) {
    launch_dirs_mode<1>(g, gr, variant, dirs_g, dirs_f, type, marks, list, cnt, s);
}

void launch_detect_only(const uint8_t* dirs_f, const uint8_t* dirs_g, const Grid& gr, int type,
                        uint8_t* marks, int* list, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_detect_only, dim3(blocks_for(gr.n, 256 * 4, 8192)), dim3(256), 0, s, dirs_f,
                       dirs_g, gr, type, marks, list, cnt);
}

void launch_apply(const int* list, int len, float* g, const float* L, uint8_t* marks, unsigned* cnt,
                  hipStream_t s) {
    if (len <= 0) return;
    hipLaunchKernelGGL(k_apply, dim3(blocks_for(len, 256, 4096)), dim3(256), 0, s, list, len, g, L,
                       marks, cnt);
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
    hipLaunchKernelGGL(k_label_final, dim3(blocks_for(n, 256 * 4, 8192)), dim3(256), 0, s, q_up, q_dn,
                       n, M, m);
}

void launch_detect_r(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* q_up, const int* q_dn,
                     const int* Mf, const int* mf, const Grid& gr, uint8_t* marks, int* list,
                     unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_detect_r, dim3(blocks_for(gr.n, 256 * 4, 8192)), dim3(256), 0, s, dirs_f,
                       dirs_g, q_up, q_dn, Mf, mf, gr, marks, list, cnt);
}

void launch_compare(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* qfu, const int* qfd,
                    const int* qgu, const int* qgd, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_compare, dim3(blocks_for(n, 256 * 4, 8192)), dim3(256), 0, s, dirs_f, dirs_g,
                       qfu, qfd, qgu, qgd, n, cnt);
}

void launch_validate_init(const float* f, const float* fhat, const float* warm, float xi, int n,
                          float* L, float* g, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_validate_init, dim3(blocks_for(n, 256 * 4, 8192)), dim3(256), 0, s, f, fhat,
                       warm, xi, n, L, g, cnt);
}

void launch_check_finite(const float* h, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 256 * 4, 8192)), dim3(256), 0, s, h, n, cnt);
}

void launch_delta(const float* g, const float* fhat, int n, float* delta, float* g_out, unsigned* cnt,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_delta, dim3(blocks_for(n, 256 * 4, 8192)), dim3(256), 0, s, g, fhat, n, delta,
                       g_out, cnt);
}

}  // namespace msz
