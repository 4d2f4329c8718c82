// msz_kernels.hip -- gfx950 kernels of the MSz correction loop (arXiv 2406.09423).
//
// Data layout in HBM (one field of n vertices, x fastest):
//   h / g / L      float32[n]
//   dirs           uint8[n]   high nibble = ascent slot, low nibble = descent slot, 0xF = self
//   cases          uint8[n]   bit t: the vertex is a C-loop case of type t (padded to 16 B)
//   marks          uint8[n]   claims of the targets edited in the current round (an
//                             edit shared by several cases is made once; padded to 16 B)
//   dirty          uint8[n]   directions to recompute after an apply (padded to 16 B)
//   M_f, m_f       int32[n]   pointer arrays of f's ascending / descending forests
//   q_up, q_dn     int32[n]   pointer arrays of g's ascending / descending forests; in
//                             both pairs a root (extremum) id as itself (>= 0), an exit
//                             of the vertex's label tile, a vertex e of the next tile on
//                             its line, as -e-1 (a label is the root at the end of the
//                             vertex's chain of exits)
//   tile_dirty     uint8      per label tile: a direction of g in it changed since its
//                             last tile pass
//   cnt            uint32[kSlots][kSlotStride] round counters; block b adds into slot
//                  b % kSlots so that no cache line takes more than a few hundred
//                  atomics per launch
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
__device__ __forceinline__ void block_add(unsigned (&v)[K], unsigned* dst, const int* idx, int nslots = kSlots,
                                          int stride = kSlotStride) {
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
        if (s) atomicAdd(dst + (blockIdx.x % nslots) * stride + idx[threadIdx.x], s);
    }
}

// One decreasing edit (Eqs. 2-6): halfway to the floor, snapped to it when
// float32 rounding would leave the value unchanged.
__device__ __forceinline__ float halve(float g, float L) {
    const float s = __fadd_rn(g, L);
    const float h = __fmul_rn(s, 0.5f);
    return h == g ? L : h;
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

// Validation of the 4-vertex group w (vector path when the group is whole).
__device__ __forceinline__ void validate_group(const float* __restrict__ f, const float* __restrict__ fhat,
                                               const float* __restrict__ warm, float xi, int n, float* __restrict__ L,
                                               float* __restrict__ g, int w, unsigned& bad) {
    if (4 * w + 3 < n) {
        const float4 f4 = reinterpret_cast<const float4*>(f)[w];
        const float4 h4 = reinterpret_cast<const float4*>(fhat)[w];
        const float fv[4] = {f4.x, f4.y, f4.z, f4.w}, hv[4] = {h4.x, h4.y, h4.z, h4.w};
        float lv[4], gv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) validate_one(fv[j], hv[j], warm, 4 * w + j, xi, lv[j], gv[j], bad);
        reinterpret_cast<float4*>(L)[w] = make_float4(lv[0], lv[1], lv[2], lv[3]);
        reinterpret_cast<float4*>(g)[w] = make_float4(gv[0], gv[1], gv[2], gv[3]);
    } else {
        for (int i = 4 * w; i < n; ++i) {
            float li, gi;
            validate_one(f[i], fhat[i], warm, i, xi, li, gi, bad);
            L[i] = li;
            g[i] = gi;
        }
    }
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

// The four C-loop predicates (Defs. 1-3) of a vertex from its packed
// directions in f (df) and g (dg): bit t set when it is a case of type t
// (0 FPmax, 1 FPmin, 2 FNmax, 3 FNmin).  The edit target of a case (Eqs. 2-5)
// is the vertex itself for FPmax and FNmin, dn_f for FPmin and up_g for FNmax.
__device__ __forceinline__ unsigned case_bits(unsigned df, unsigned dg) {
    const unsigned uf = df >> 4, nf = df & 15u, ug = dg >> 4, ng = dg & 15u;
    const unsigned c0 = (ug == kSelf) & (uf != kSelf);   // FPmax
    const unsigned c1 = (ng == kSelf) & (nf != kSelf);   // FPmin
    const unsigned c2 = (uf == kSelf) & (ug != kSelf);   // FNmax
    const unsigned c3 = (nf == kSelf) & (ng != kSelf);   // FNmin
    return c0 | (c1 << 1) | (c2 << 2) | (c3 << 3);
}

// Four packed direction bytes at once (byte k = vertex i0 + k): bit 4 of
// byte k is set when that vertex's ascent (hi) or descent (lo) nibble is the
// self slot 0xF.  A nibble y' = 15 - nibble is 0 exactly then, and
// y' + 15 < 32 carries into bit 4 exactly when y' > 0; no byte carries into
// the next.
__device__ __forceinline__ unsigned hi_self4(unsigned d) {
    return ~(((~d >> 4) & 0x0F0F0F0Fu) + 0x0F0F0F0Fu) & 0x10101010u;
}
__device__ __forceinline__ unsigned lo_self4(unsigned d) {
    return ~((~d & 0x0F0F0F0Fu) + 0x0F0F0F0Fu) & 0x10101010u;
}

// case_bits of four vertices at once (byte k = vertex k) from their packed
// directions in f (df4) and g (dg4); a byte of 0xFF in both (a vertex outside
// the grid) has no case.  Adds the count of each type to c.
__device__ __forceinline__ unsigned cases4(unsigned df4, unsigned dg4, unsigned (&c)[4]) {
    const unsigned ug = hi_self4(dg4), uf = hi_self4(df4), ng = lo_self4(dg4), nf = lo_self4(df4);
    const unsigned fpmax = ug & ~uf, fpmin = ng & ~nf, fnmax = uf & ~ug, fnmin = nf & ~ng;
    c[0] += __popc(fpmax);
    c[1] += __popc(fpmin);
    c[2] += __popc(fnmax);
    c[3] += __popc(fnmin);
    // bit 4 of each byte moves to bit t of the same byte
    return (fpmax >> 4) | (fpmin >> 3) | (fnmax >> 2) | (fnmin >> 1);
}

// Per-vertex byte arrays written by the full direction pass of g (MODE 1):
// the case bits, and the dirty flags and claim marks of the incremental
// refresh, which the full pass clears.
struct CaseArrays {
    uint8_t *cases, *dirty, *marks;
};

// --------------------------------------------------- steepest directions ---
//
// Work item = a 64 x TY column of ZC planes (2D: one 64 x TY tile).  A block
// is persistent: it walks a contiguous range of work items (XCD-aware, so the
// halos of neighbouring items stay in the same L2) as one stream of planes.
// Each plane, with a one-vertex halo (NaN outside the grid, so it never wins a
// comparison), is loaded into registers one step ahead, stored into a ring of
// three LDS planes, and the middle plane is then computed: a thread owns four
// x-consecutive vertices of TY/16 rows.  Loads are issued as a batch before
// the previous plane is computed, which keeps HBM busy.
//
// MODE 0: write dirs only.  MODE 1: also write the case bits of every vertex
// against dirs_f, count each type and clear the dirty flags and marks.

// Maps the hardware block id to a tile so that consecutive tiles land on the
// same XCD (blocks are dealt to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, k = b & 7;
    return k * q + min(k, r) + (b >> 3);
}

// Running steepest ascent / descent of one vertex.  Neighbours are fed in
// increasing order of |id - centre| on each side of the centre: first the
// ones with a smaller id (below), then the ones with a larger id (above).
// The order (value, id) then needs no id comparison: a below-centre
// neighbour must be strictly higher to become the ascent and wins descent
// ties (it has the smaller id); an above-centre neighbour wins ascent ties
// and must be strictly lower to become the descent.  Which neighbour ids are
// smaller or larger does not depend on the grid size (checked for all grids
// up to 6x6 and 5x5x5; for larger ones the offsets only grow apart).  NaN
// (outside the grid) fails every comparison and is never chosen.
struct Steepest {
    float uv, dv;
    unsigned us, ds;
    __device__ __forceinline__ void below(float w, unsigned slot) {
        if (w > uv) uv = w, us = slot;
        if (w <= dv) dv = w, ds = slot;
    }
    __device__ __forceinline__ void above(float w, unsigned slot) {
        if (w >= uv) uv = w, us = slot;
        if (w < dv) dv = w, ds = slot;
    }
};

// LDS plane layout: rows of W = 72 floats; column 4 + c holds x = x0 + c
// (c = 0..63), column 3 the left halo x0 - 1, column 68 the right halo
// x0 + 64, so every 4-vertex group starts on a 16-byte boundary.  H = TY + 2
// rows (y0 - 1 .. y0 + TY).  A plane is loaded as 16 float4 per row plus two
// halo floats per row.
template <int NDIM, int TY, int ZC>
struct DirsGeom {
    static constexpr int W = 72, H = TY + 2, P = W * H, RPT = TY / 16;
    static constexpr int NV = 16 * H, NH = 2 * H;               // float4 and halo loads per plane
    static constexpr int LV = (NV + 255) / 256, LH = (NH + 255) / 256;
    static constexpr int NP = NDIM == 3 ? 3 : 1;     // LDS ring of planes
    static constexpr int ZCH = NDIM == 3 ? ZC : 1;   // planes computed per work item
    int tiles_x, tiles_y, tiles_z;
    __device__ __forceinline__ explicit DirsGeom(const Grid& gr)
        : tiles_x((gr.nx + kTileX - 1) / kTileX),
          tiles_y((gr.ny + TY - 1) / TY),
          tiles_z(NDIM == 3 ? (gr.nz + ZCH - 1) / ZCH : 1) {}
    __device__ __forceinline__ int items() const { return tiles_x * tiles_y * tiles_z; }
    __device__ __forceinline__ void origin(int it, int& x0, int& y0, int& z0) const {
        x0 = (it % tiles_x) * kTileX;
        y0 = ((it / tiles_x) % tiles_y) * TY;
        z0 = NDIM == 3 ? (it / (tiles_x * tiles_y)) * ZCH : 0;
    }
    // planes streamed for item it: z0 - 1 .. z0 + zc in 3D, the single plane in 2D
    __device__ __forceinline__ int planes(const Grid& gr, int it) const {
        if constexpr (NDIM == 3) {
            const int z0 = (it / (tiles_x * tiles_y)) * ZCH;
            return min(ZCH, gr.nz - z0) + 2;
        }
        return 1;
    }
};

// Registers holding one plane between its load and its LDS store.
template <int NDIM, int TY, int ZC>
struct PlaneRegs {
    using G = DirsGeom<NDIM, TY, ZC>;
    float4 v[G::LV];
    float h[G::LH];
    unsigned d[G::RPT];  // MODE 1: dirs_f words of the plane computed next
};

// A work item's origin, plane count and whether all of it and its halo lie
// inside the grid (then no load or store needs a bounds check).  Uniform
// over the block.
struct ItemPos {
    int x0, y0, z0, planes;
    bool interior;
};

template <int NDIM, int TY, int ZC>
__device__ __forceinline__ ItemPos item_pos(const DirsGeom<NDIM, TY, ZC>& geo, const Grid& gr, int it, bool vec4) {
    ItemPos p;
    geo.origin(it, p.x0, p.y0, p.z0);
    p.planes = geo.planes(gr, it);
    const bool zin = NDIM == 2 || (p.z0 >= 1 && p.z0 + ZC < gr.nz);
    p.interior = vec4 && zin && p.x0 >= 1 && p.x0 + kTileX < gr.nx && p.y0 >= 1 && p.y0 + TY < gr.ny;
    return p;
}

// Issues the loads of plane j of the item at pos into registers (and, in
// MODE 1, the dirs_f words of the plane that is computed once this one is in
// LDS).  Outside the grid a value is NaN, which never wins a comparison.
// vec4: rows start 16-byte aligned (nx % 4 == 0 and an aligned base), so
// whole in-grid groups of four are one dwordx4 load.
template <int NDIM, int TY, int ZC, int MODE>
__device__ __forceinline__ void dirs_load(const float* __restrict__ h, const uint8_t* __restrict__ dirs_f,
                                          const Grid& gr, const ItemPos& pos, bool vec4, int j,
                                          PlaneRegs<NDIM, TY, ZC>& pr) {
    using G = DirsGeom<NDIM, TY, ZC>;
    const int x0 = pos.x0, y0 = pos.y0;
    const int z = NDIM == 3 ? pos.z0 - 1 + j : 0;
    const float* plane = h + static_cast<long>(z) * gr.nxy;
    const float nan = __builtin_nanf("");
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int zc = NDIM == 3 ? z - 1 : 0;
    if (pos.interior) {
#pragma unroll
        for (int k = 0; k < G::LV; ++k) {
            const int u = threadIdx.x + 256 * k;
            float4 v = make_float4(nan, nan, nan, nan);
            if (G::NV % 256 == 0 || u < G::NV)
                v = *reinterpret_cast<const float4*>(plane + static_cast<long>(gr.nx) * (y0 + (u >> 4) - 1) + x0 +
                                                     4 * (u & 15));
            pr.v[k] = v;
        }
#pragma unroll
        for (int k = 0; k < G::LH; ++k) {
            const int u = threadIdx.x + 256 * k;
            float v = nan;
            if (u < G::NH) v = plane[static_cast<long>(gr.nx) * (y0 + (u >> 1) - 1) + ((u & 1) ? x0 + kTileX : x0 - 1)];
            pr.h[k] = v;
        }
        if constexpr (MODE == 1) {
            if (NDIM == 2 || j >= 2) {
#pragma unroll
                for (int q = 0; q < G::RPT; ++q)
                    pr.d[q] = *reinterpret_cast<const unsigned*>(
                        dirs_f + static_cast<long>(zc) * gr.nxy + static_cast<long>(gr.nx) * (y0 + ty + 16 * q) + x0 + 4 * tx);
            }
        }
        return;
    }
    const bool zin = z >= 0 && z < gr.nz;
#pragma unroll
    for (int k = 0; k < G::LV; ++k) {
        const int u = threadIdx.x + 256 * k;
        const int r = u >> 4, x = x0 + 4 * (u & 15), y = y0 + r - 1;
        float4 v = make_float4(nan, nan, nan, nan);
        if (u < G::NV && zin && y >= 0 && y < gr.ny && x < gr.nx) {
            const float* src = plane + static_cast<long>(gr.nx) * y + x;
            if (vec4 && x + 3 < gr.nx) {
                v = *reinterpret_cast<const float4*>(src);
            } else {
                v.x = src[0];
                if (x + 1 < gr.nx) v.y = src[1];
                if (x + 2 < gr.nx) v.z = src[2];
                if (x + 3 < gr.nx) v.w = src[3];
            }
        }
        pr.v[k] = v;
    }
#pragma unroll
    for (int k = 0; k < G::LH; ++k) {
        const int u = threadIdx.x + 256 * k;
        const int r = u >> 1, x = (u & 1) ? x0 + kTileX : x0 - 1, y = y0 + r - 1;
        float v = nan;
        if (u < G::NH && zin && y >= 0 && y < gr.ny && x >= 0 && x < gr.nx)
            v = plane[static_cast<long>(gr.nx) * y + x];
        pr.h[k] = v;
    }
    if constexpr (MODE == 1) {
        const bool dvec = (gr.nx & 3) == 0;
        const bool zok = NDIM == 3 ? (j >= 2 && zc < gr.nz) : true;
#pragma unroll
        for (int q = 0; q < G::RPT; ++q) {
            const int y = y0 + ty + 16 * q, xa = x0 + tx * 4;
            const long i0 = static_cast<long>(zc) * gr.nxy + static_cast<long>(gr.nx) * y + xa;
            unsigned d = 0xFFFFFFFFu;
            if (zok && y < gr.ny) {
                if (dvec && xa + 3 < gr.nx) {
                    d = *reinterpret_cast<const unsigned*>(dirs_f + i0);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (xa + k < gr.nx) d = (d & ~(0xFFu << (8 * k))) | (static_cast<unsigned>(dirs_f[i0 + k]) << (8 * k));
                }
            }
            pr.d[q] = d;
        }
    }
}

// Stores a loaded plane into its LDS slot.
template <int NDIM, int TY, int ZC>
__device__ __forceinline__ void dirs_store(float* slot, const PlaneRegs<NDIM, TY, ZC>& pr) {
    using G = DirsGeom<NDIM, TY, ZC>;
#pragma unroll
    for (int k = 0; k < G::LV; ++k) {
        const int u = threadIdx.x + 256 * k;
        if (u < G::NV) *reinterpret_cast<float4*>(slot + (u >> 4) * G::W + 4 + 4 * (u & 15)) = pr.v[k];
    }
#pragma unroll
    for (int k = 0; k < G::LH; ++k) {
        const int u = threadIdx.x + 256 * k;
        if (u < G::NH) slot[(u >> 1) * G::W + ((u & 1) ? 4 + kTileX : 3)] = pr.h[k];
    }
}

// Six consecutive LDS values of a row around a 4-vertex group: the group
// (one 16-byte read) and its left and right neighbours.
struct Row6 {
    float l, a, b, c, d, r;
    __device__ __forceinline__ explicit Row6(const float* p) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        l = p[-1];
        a = v.x, b = v.y, c = v.z, d = v.w;
        r = p[4];
    }
    // value at column offset o in -1..4 (o is a compile-time constant after unrolling)
    __device__ __forceinline__ float at(int o) const {
        return o < 0 ? l : o == 0 ? a : o == 1 ? b : o == 2 ? c : o == 3 ? d : r;
    }
};

// Directions (and, in MODE 1, detection) of plane z of the item at pos, from
// the LDS planes C (z), A (z + 1) and B (z - 1).
template <int NDIM, int TY, int ZC, int MODE>
__device__ __forceinline__ void dirs_compute(const float* C, const float* A, const float* B, const Grid& gr,
                                             const ItemPos& pos, int z,
                                             const unsigned (&df4)[DirsGeom<NDIM, TY, ZC>::RPT],
                                             uint8_t* __restrict__ dirs_out, const CaseArrays& ca,
                                             unsigned (&c)[4]) {
    using G = DirsGeom<NDIM, TY, ZC>;
    constexpr int W = G::W;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const bool vec4 = (gr.nx & 3) == 0;
#pragma unroll
    for (int q = 0; q < G::RPT; ++q) {
        const int y = pos.y0 + ty + 16 * q, xa = pos.x0 + tx * 4, r = ty + 16 * q + 1;
        const long i0 = static_cast<long>(z) * gr.nxy + static_cast<long>(gr.nx) * y + xa;
        const bool full = pos.interior || (vec4 && xa + 3 < gr.nx && y < gr.ny);
        const int col = 4 + 4 * tx;
        const Row6 cm(C + (r - 1) * W + col), c0(C + r * W + col), cp(C + (r + 1) * W + col);
        Row6 bm = c0, b0 = c0, a0 = c0, ap = c0;
        if constexpr (NDIM == 3) {
            bm = Row6(B + (r - 1) * W + col);
            b0 = Row6(B + r * W + col);
            a0 = Row6(A + r * W + col);
            ap = Row6(A + (r + 1) * W + col);
        }
        unsigned out4 = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool valid = pos.interior || (xa + k < gr.nx && y < gr.ny);
            if (valid) {
                const float v = c0.at(k);
                Steepest b{v, v, kSelf, kSelf};
                // below-centre ids, nearest first, then above-centre ids, nearest first
                b.below(c0.at(k - 1), 1);
                b.below(cm.at(k), 3);
                b.below(cm.at(k - 1), 5);
                if constexpr (NDIM == 3) {
                    b.below(b0.at(k), 7);
                    b.below(b0.at(k - 1), 9);
                    b.below(bm.at(k), 11);
                    b.below(bm.at(k - 1), 13);
                }
                b.above(c0.at(k + 1), 0);
                b.above(cp.at(k), 2);
                b.above(cp.at(k + 1), 4);
                if constexpr (NDIM == 3) {
                    b.above(a0.at(k), 6);
                    b.above(a0.at(k + 1), 8);
                    b.above(ap.at(k), 10);
                    b.above(ap.at(k + 1), 12);
                }
                const unsigned packed = (b.us << 4) | b.ds;
                out4 = (out4 & ~(0xFFu << (8 * k))) | (packed << (8 * k));
                if (!full) dirs_out[i0 + k] = static_cast<uint8_t>(packed);
            }
        }
        if (full) *reinterpret_cast<unsigned*>(dirs_out + i0) = out4;
        if constexpr (MODE == 1) {
            // 32-bit offsets (n < 2^31) keep the three stores on one address register
            const unsigned u0 = static_cast<unsigned>(i0);
            const unsigned cw = cases4(df4[q], out4, c);
            if (full) {
                *reinterpret_cast<unsigned*>(ca.cases + u0) = cw;
                *reinterpret_cast<unsigned*>(ca.dirty + u0) = 0u;
                *reinterpret_cast<unsigned*>(ca.marks + u0) = 0u;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (pos.interior || (xa + k < gr.nx && y < gr.ny)) {
                        ca.cases[u0 + k] = static_cast<uint8_t>(cw >> (8 * k));
                        ca.dirty[u0 + k] = 0;
                        ca.marks[u0 + k] = 0;
                    }
            }
        }
    }
}

// Stream of planes over the work items `range` (one item, or a persistent
// block's whole range), each plane prefetched in registers one step ahead.
// sm: LDS of NP * P floats.
template <int NDIM, int TY, int ZC, int MODE>
__device__ __forceinline__ void dirs_stream(const float* __restrict__ h, const Grid& gr, ItemRange range,
                                            uint8_t* __restrict__ dirs_out, const uint8_t* __restrict__ dirs_f,
                                            const CaseArrays& ca, float* sm, unsigned (&c)[4]) {
    using G = DirsGeom<NDIM, TY, ZC>;
    const G geo(gr);
    const bool vec4 = (gr.nx & 3) == 0 && (reinterpret_cast<uintptr_t>(h) & 15u) == 0 &&
                      (MODE == 0 || (reinterpret_cast<uintptr_t>(dirs_f) & 3u) == 0) &&
                      (reinterpret_cast<uintptr_t>(dirs_out) & 3u) == 0;
    PlaneRegs<NDIM, TY, ZC> pr;
    int it = range.first, j = 0;
    ItemPos pos{};
    if (it < range.hi) {
        pos = item_pos(geo, gr, it, vec4);
        dirs_load<NDIM, TY, ZC, MODE>(h, dirs_f, gr, pos, vec4, 0, pr);
    }
    int ring = 0;  // LDS slot of the plane held in registers
    while (it < range.hi) {
        dirs_store<NDIM, TY, ZC>(sm + ring * G::P, pr);
        unsigned df4[G::RPT];
#pragma unroll
        for (int q = 0; q < G::RPT; ++q) df4[q] = pr.d[q];
        __syncthreads();
        // advance the stream and prefetch the next plane while this one is computed
        const ItemPos cur = pos;
        const int cur_j = j, cur_ring = ring;
        if (++j == pos.planes) {
            j = 0;
            it += range.stride;
            if (it < range.hi) pos = item_pos(geo, gr, it, vec4);
        }
        ring = G::NP == 3 ? (ring + 1) % 3 : 0;
        if (it < range.hi) dirs_load<NDIM, TY, ZC, MODE>(h, dirs_f, gr, pos, vec4, j, pr);
        if (NDIM == 2 || cur_j >= 2) {
            const int z = NDIM == 3 ? cur.z0 + cur_j - 2 : 0;
            const float* A = sm + cur_ring * G::P;                             // plane z + 1
            const float* C = sm + (G::NP == 3 ? (cur_ring + 2) % 3 : 0) * G::P; // plane z
            const float* B = sm + (G::NP == 3 ? (cur_ring + 1) % 3 : 0) * G::P; // plane z - 1
            dirs_compute<NDIM, TY, ZC, MODE>(C, A, B, gr, cur, z, df4, dirs_out, ca, c);
        }
        __syncthreads();  // the slot written next is the oldest plane
    }
}

// Directions only (msz_labels, msz_count_false and the network features).
template <int NDIM, int TY, int ZC>
__global__ void __launch_bounds__(256) k_dirs(const float* __restrict__ h, Grid gr, uint8_t* __restrict__ dirs_out) {
    using G = DirsGeom<NDIM, TY, ZC>;
    static_assert(TY % 16 == 0, "a thread row covers 16 tile rows");
    __shared__ __align__(16) float sm[G::NP * G::P];
    unsigned c[4] = {0u, 0u, 0u, 0u};
    const CaseArrays none{nullptr, nullptr, nullptr};
    dirs_stream<NDIM, TY, ZC, 0>(h, gr, xcd_items(G(gr).items()), dirs_out, nullptr, none, sm, c);
}

// ---------------------------------------------------------------- apply ---
//
// One decreasing edit (Eqs. 2-6) per target and round.  The correction loop
// keeps, besides the directions of g, a case byte per vertex (case_bits), so
// an apply step needs no detection pass: it scans the case bytes for the
// current type and edits the targets (the R loop edits the troublemakers'
// targets in the detection step itself).  Every edited vertex and, when its value changed, every
// neighbour is flagged dirty: only their directions can have changed, and the
// refresh step recomputes exactly those (the synchronous round is unchanged,
// so results are identical to a full recomputation).

// Slot deltas in the order of the neighbour table at the top of this file,
// as (d + 1) in two bits per slot (slot 0 lowest; slots 14 and 15, the self
// slot, are 0, 0, 0): decoded in registers, where a table indexed by a
// per-lane slot would be a memory load per lookup.
constexpr int kSlotDX[14] = {1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1};
constexpr int kSlotDY[14] = {0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kSlotDZ[14] = {0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr unsigned pack_slots(const int (&d)[14]) {
    unsigned p = 0;
    for (int s = 0; s < 16; ++s) p |= static_cast<unsigned>((s < 14 ? d[s] : 0) + 1) << (2 * s);
    return p;
}
constexpr unsigned kPackDX = pack_slots(kSlotDX), kPackDY = pack_slots(kSlotDY), kPackDZ = pack_slots(kSlotDZ);

__device__ __forceinline__ void slot_delta(unsigned s, int& dx, int& dy, int& dz) {
    dx = static_cast<int>((kPackDX >> (2 * s)) & 3u) - 1;
    dy = static_cast<int>((kPackDY >> (2 * s)) & 3u) - 1;
    dz = static_cast<int>((kPackDZ >> (2 * s)) & 3u) - 1;
}

// Linear id offset of neighbour slot s (0 for the self slot); the same as
// gr.off[s], computed in registers for a per-lane slot.
__device__ __forceinline__ int slot_offset(const Grid& gr, unsigned s) {
    int dx, dy, dz;
    slot_delta(s, dx, dy, dz);
    return dx + gr.nx * dy + gr.nxy * dz;
}

// Whether neighbour slot s of the vertex at (x, y, z) lies in the grid.
template <int NDIM>
__device__ __forceinline__ bool slot_in_grid(const Grid& gr, int x, int y, int z, int s) {
    int dx, dy, dz;
    slot_delta(s, dx, dy, dz);
    const bool in2 = x + dx >= 0 && x + dx < gr.nx && y + dy >= 0 && y + dy < gr.ny;
    return NDIM == 2 ? in2 : in2 && z + dz >= 0 && z + dz < gr.nz;
}

// The refresh flags: one byte per vertex, and per kEngChunk vertices a word
// that is set when some flag of the chunk may be (chunk: NULL where the
// summaries are not kept), so that a refresh reads only the chunks an edit
// touched.
struct Dirty {
    uint8_t* v;
    unsigned* chunk;
    __device__ __forceinline__ void mark(int i) const {
        v[i] = 1;
        if (chunk) chunk[i >> kEngChunkShift] = 1u;
    }
};

// Halves g[t] once, from its value old and floor lt as read by the caller;
// flags t (so the refresh clears its mark) and, if the value changed, its
// neighbours.
template <int NDIM>
__device__ __forceinline__ void edit_value(float* __restrict__ g, const Dirty& dirty, const Grid& gr,
                                           int t, float old, float lt, unsigned& changed) {
    const float nv = halve(old, lt);
    dirty.mark(t);
    if (nv == old) return;
    g[t] = nv;
    ++changed;
    const int x = t % gr.nx, y = (t / gr.nx) % gr.ny, z = NDIM == 3 ? t / gr.nxy : 0;
    constexpr int NS = NDIM == 3 ? 14 : 6;
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (slot_in_grid<NDIM>(gr, x, y, z, s)) dirty.mark(t + gr.off[s]);
}

template <int NDIM>
__device__ __forceinline__ void edit_vertex(float* __restrict__ g, const float* __restrict__ L,
                                            const Dirty& dirty, const Grid& gr, int t, unsigned& changed) {
    edit_value<NDIM>(g, dirty, gr, t, g[t], L[t], changed);
}

// Edits target t unless another case of the same step already has: the first
// to set t's mark (an atomic OR on its word) edits it.  The mark is cleared by
// the refresh that follows (t is flagged by the edit).  g[t] and L[t] are read
// alongside the atomic (one memory round trip, not two): within a step only
// the winner writes g[t], so the value read is the round's.
template <int NDIM>
__device__ __forceinline__ void claim_edit(uint8_t* __restrict__ marks, float* __restrict__ g,
                                           const float* __restrict__ L, const Dirty& dirty,
                                           const Grid& gr, int t, unsigned& changed) {
    const unsigned bit = 1u << (8 * (t & 3));
    // relaxed workgroup-scope atomic loads: plain cached loads that the
    // compiler keeps ahead of the atomic instead of sinking them into the
    // winner's branch
    const float old = __hip_atomic_load(g + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const float lt = __hip_atomic_load(L + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if ((atomicOr(reinterpret_cast<unsigned*>(marks + (t & ~3)), bit) & bit) == 0u)
        edit_value<NDIM>(g, dirty, gr, t, old, lt, changed);
}

// Preemptive edit (the preemptive mode of Sec. 6.1): halves g[t] from
// whatever value it holds when read, with no claim.  Cases that share a
// target race: those that read the same value write the same result (one
// edit survives; the lost ones come back as cases in a later round), and one
// that reads another's result halves it again.  Every value written is a
// halving of a value no larger than the round's snapshot, so a round still
// lowers each target it changes and the loop ends as the synchronous one does.
template <int NDIM>
__device__ __forceinline__ void preempt_edit(float* __restrict__ g, const float* __restrict__ L,
                                             const Dirty& dirty, const Grid& gr, int t, unsigned& changed) {
    const float old = __hip_atomic_load(g + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float nv = halve(old, L[t]);
    dirty.mark(t);
    if (nv == old) return;
    __hip_atomic_store(g + t, nv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++changed;
    const int x = t % gr.nx, y = (t / gr.nx) % gr.ny, z = NDIM == 3 ? t / gr.nxy : 0;
    constexpr int NS = NDIM == 3 ? 14 : 6;
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (slot_in_grid<NDIM>(gr, x, y, z, s)) dirty.mark(t + gr.off[s]);
}

// A shared target's edit: claimed (synchronous rounds) or preemptive.
template <int NDIM>
__device__ __forceinline__ void target_edit(bool preempt, uint8_t* __restrict__ marks, float* __restrict__ g,
                                            const float* __restrict__ L, const Dirty& dirty,
                                            const Grid& gr, int t, unsigned& changed) {
    if (preempt) preempt_edit<NDIM>(g, L, dirty, gr, t, changed);
    else claim_edit<NDIM>(marks, g, L, dirty, gr, t, changed);
}

// --------------------------------------------------------------- labels ---
//
// Pointer jumping along the forests of steepest ascent and descent (Sec. 6.2).
// Stage 1 resolves each 4096-vertex tile inside LDS: every vertex ends up
// pointing at either the extremum it reaches inside its tile (stored as its
// id) or the first vertex e outside the tile on its integral line (stored as
// -e-1).  Such exit targets lie on the face layer of their own tile.  A label
// is then the end of a short chain of exits (on the fields here a tile exit
// leads on through another tile a quarter of the time): follow_root walks it.
// The correction loop follows the chains where it needs labels (a few
// gathers per hundred vertices).  msz_labels and msz_count_false first
// compress the exit targets' pointers to their roots (each thread walks its
// own chain, writing back every step; any value read is an ancestor, so no
// barrier is needed and each walk strictly advances).

// Label tiles of 4096 vertices, wide in x: a tile row fills whole 128-byte
// lines of the int32 arrays the label passes stream (16^3 tiles used half of
// each line and fetched 2.8 times the pass's bytes); measured best among
// 16x16x16, 32x16x8, 32x32x4, 64x16x4, 64x8x8 and 128x8x4 (3D) and 64x64,
// 128x32 and 256x16 (2D).
template <int NDIM>
struct LabelTile;
template <>
struct LabelTile<2> {
    static constexpr int X = 128, Y = 32, Z = 1;
};
template <>
struct LabelTile<3> {
    static constexpr int X = 64, Y = 8, Z = 8;
};

__host__ __device__ __forceinline__ int label_tiles_of(const Grid& gr) {
    if (gr.ndim == 2) {
        using T = LabelTile<2>;
        return ((gr.nx + T::X - 1) / T::X) * ((gr.ny + T::Y - 1) / T::Y);
    }
    using T = LabelTile<3>;
    return ((gr.nx + T::X - 1) / T::X) * ((gr.ny + T::Y - 1) / T::Y) * ((gr.nz + T::Z - 1) / T::Z);
}

// The stored pointer of a tile-pass terminal a (tile origin X0, Y0, Z0): an
// exit code -e-1 as it is, an extremum's local code as its global id.  (A
// non-negative a, a local index, cannot remain after the jumping; it would
// name an in-tile ancestor.)
template <int NDIM>
__device__ __forceinline__ int tile_term_global(const Grid& gr, int X0, int Y0, int Z0, int a) {
    using T = LabelTile<NDIM>;
    if (a < 0 && a >= -gr.n) return a;
    const int l = a < 0 ? -a - 1 - gr.n : a;
    return X0 + l % T::X + gr.nx * (Y0 + (l / T::X) % T::Y) + gr.nxy * (Z0 + l / (T::X * T::Y));
}

// Follows K chains of exits from stored pointers y[k] to their roots, one
// level per pass, so that the gathers of a pass are in flight together (y[k]
// in q_up when k is even, in q_dn when odd; entries already >= 0 stay).  With
// S < K, the entries from S on belong to a second forest, r_up / r_dn, whose
// chains are followed in the same passes.  Every chain of the forest ends at
// an extremum within finitely many tiles.  hops counts the gathers; the pass
// cap only guards against corrupted input and sets bad.
constexpr int kMaxChain = 1 << 20;

template <int K, int S = K>
__device__ __forceinline__ void follow_roots(const int* q_up, const int* q_dn, int (&y)[K], unsigned& bad,
                                             unsigned& hops, const int* r_up = nullptr, const int* r_dn = nullptr) {
    for (int pass = 0;; ++pass) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= y[k] < 0;
        if (!any) return;
        if (pass == kMaxChain) {
            bad = kErrWalk;
#pragma unroll
            for (int k = 0; k < K; ++k) y[k] = max(y[k], 0);
            return;
        }
        // unconditional loads (a finished chain reads entry 0, one line for
        // the whole wave), so that all K are issued before the first wait
        int z[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            z[k] = (k < S ? ((k & 1) ? q_dn : q_up) : ((k & 1) ? r_dn : r_up))[y[k] < 0 ? -y[k] - 1 : 0];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            hops += y[k] < 0;
            y[k] = y[k] < 0 ? z[k] : y[k];
        }
    }
}

// One label tile; su, sd: LDS arrays of the tile's vertex count.  The caller
// separates consecutive tiles of one block with a barrier.
//
// Thread t owns the 4-vertex row groups starting at l = 4 t + 1024 k and
// keeps their pointers in registers; the LDS copy is what other threads read.
// Terminal pointers are negative: an exit e as -e-1 (in -n .. -1), an in-tile
// extremum with local index l as -(n + l) - 1 (below -n; n + 4096 < 2^31).
template <int NDIM>
__device__ __forceinline__ void label_tile_body(const uint8_t* __restrict__ dirs, const Grid& gr, int tile,
                                                int* __restrict__ q_up, int* __restrict__ q_dn, int* su, int* sd) {
    using T = LabelTile<NDIM>;
    constexpr int NT = T::X * T::Y * T::Z;
    constexpr int G = NT / 1024;  // row groups per thread

    const int tx_n = (gr.nx + T::X - 1) / T::X;
    const int ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int bx = tile % tx_n, by = (tile / tx_n) % ty_n, bz = tile / (tx_n * ty_n);
    const int X0 = bx * T::X, Y0 = by * T::Y, Z0 = bz * T::Z;

    const bool vec4 = (gr.nx & 3) == 0;
    int pu[G][4], pd[G][4];
    unsigned d4[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {  // the direction words first, all in flight together
        const int l0 = 4 * threadIdx.x + 1024 * k;
        const int lx0 = l0 % T::X, ly = (l0 / T::X) % T::Y, lz = l0 / (T::X * T::Y);
        const int xa = X0 + lx0, y = Y0 + ly, z = Z0 + lz;
        const bool row_in = y < gr.ny && z < gr.nz;
        const int i0 = xa + gr.nx * y + gr.nxy * z;
        d4[k] = 0xFFFFFFFFu;
        if (row_in && vec4 && xa + 3 < gr.nx) {
            d4[k] = *reinterpret_cast<const unsigned*>(dirs + i0);
        } else if (row_in) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (xa + j < gr.nx)
                    d4[k] = (d4[k] & ~(0xFFu << (8 * j))) | (static_cast<unsigned>(dirs[i0 + j]) << (8 * j));
        }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int l0 = 4 * threadIdx.x + 1024 * k;
        const int lx0 = l0 % T::X, ly = (l0 / T::X) % T::Y, lz = l0 / (T::X * T::Y);
        const int xa = X0 + lx0, y = Y0 + ly, z = Z0 + lz;
        const bool row_in = y < gr.ny && z < gr.nz;
        const int i0 = xa + gr.nx * y + gr.nxy * z;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int lx = lx0 + j;
            int p[2] = {-1, -1};
            if (row_in && xa + j < gr.nx) {
                const int i = i0 + j;
                const unsigned d = (d4[k] >> (8 * j)) & 0xFFu;
                const unsigned s2[2] = {d >> 4, d & 15u};
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const unsigned s = s2[w];
                    if (s == kSelf) {
                        p[w] = -(gr.n + lx + T::X * (ly + T::Y * lz)) - 1;
                    } else {
                        int dx, dy, dz;
                        slot_delta(s, dx, dy, dz);
                        const int ax = lx + dx, ay = ly + dy, az = lz + dz;
                        if (ax >= 0 && ax < T::X && ay >= 0 && ay < T::Y && az >= 0 && az < T::Z)
                            p[w] = ax + T::X * (ay + T::Y * az);
                        else
                            p[w] = -(i + slot_offset(gr, s)) - 1;
                    }
                }
            }
            pu[k][j] = p[0];
            pd[k][j] = p[1];
        }
        *reinterpret_cast<int4*>(su + l0) = make_int4(pu[k][0], pu[k][1], pu[k][2], pu[k][3]);
        *reinterpret_cast<int4*>(sd + l0) = make_int4(pd[k][0], pd[k][1], pd[k][2], pd[k][3]);
    }
    __syncthreads();
    // Pointer jumping in LDS: each thread replaces each of its non-terminal
    // pointers by the pointer stored at its target, then publishes a group's
    // four entries with one 16-byte write.  Any entry read is an ancestor of
    // the reader on its integral line (entries only ever move up their
    // forest), so no barrier is needed between jumps and every jump makes
    // progress; a pointer needs at most one jump per vertex of its in-tile
    // path.  A group is skipped once the whole wave's copies of it are
    // terminal; otherwise its eight reads are issued together, branch-free
    // (a terminal pointer reads entry 0 and keeps its value).
    for (int iter = 0; iter < NT; ++iter) {
        bool pending = false;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            bool live = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) live |= (pu[k][j] & pd[k][j]) >= 0;  // either is non-terminal
            if (!__any(live)) continue;
            int nu[4], nd[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                nu[j] = su[max(pu[k][j], 0)];
                nd[j] = sd[max(pd[k][j], 0)];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                pu[k][j] = pu[k][j] >= 0 ? nu[j] : pu[k][j];
                pd[k][j] = pd[k][j] >= 0 ? nd[j] : pd[k][j];
                pending |= (pu[k][j] & pd[k][j]) >= 0;
            }
            const int l0 = 4 * threadIdx.x + 1024 * k;
            *reinterpret_cast<int4*>(su + l0) = make_int4(pu[k][0], pu[k][1], pu[k][2], pu[k][3]);
            *reinterpret_cast<int4*>(sd + l0) = make_int4(pd[k][0], pd[k][1], pd[k][2], pd[k][3]);
        }
        if (!pending) break;
    }
    // Every in-tile path is shorter than the tile, so all pointers are terminal
    // here: an exit keeps its code, an extremum becomes its id.
    auto global_of = [&](int a) { return tile_term_global<NDIM>(gr, X0, Y0, Z0, a); };
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int l0 = 4 * threadIdx.x + 1024 * k;
        const int lx0 = l0 % T::X, ly = (l0 / T::X) % T::Y, lz = l0 / (T::X * T::Y);
        const int xa = X0 + lx0, y = Y0 + ly, z = Z0 + lz;
        if (y >= gr.ny || z >= gr.nz) continue;
        const int i0 = xa + gr.nx * y + gr.nxy * z;
        if (vec4 && xa + 3 < gr.nx) {
            *reinterpret_cast<int4*>(q_up + i0) =
                make_int4(global_of(pu[k][0]), global_of(pu[k][1]), global_of(pu[k][2]), global_of(pu[k][3]));
            *reinterpret_cast<int4*>(q_dn + i0) =
                make_int4(global_of(pd[k][0]), global_of(pd[k][1]), global_of(pd[k][2]), global_of(pd[k][3]));
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (xa + j < gr.nx) {
                    q_up[i0 + j] = global_of(pu[k][j]);
                    q_dn[i0 + j] = global_of(pd[k][j]);
                }
        }
    }
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_label_tile(const uint8_t* __restrict__ dirs, Grid gr,
                                                    int* __restrict__ q_up,
                                                    int* __restrict__ q_dn) {
    constexpr int NT = LabelTile<NDIM>::X * LabelTile<NDIM>::Y * LabelTile<NDIM>::Z;
    __shared__ __align__(16) int su[NT];
    __shared__ __align__(16) int sd[NT];
    label_tile_body<NDIM>(dirs, gr, xcd_logical_block(blockIdx.x, gridDim.x), q_up, q_dn, su, sd);
}

// Number of face-layer vertices of a full label tile.
template <int NDIM>
__host__ __device__ constexpr int face_count() {
    using T = LabelTile<NDIM>;
    return NDIM == 2 ? 2 * T::X + 2 * (T::Y - 2)
                     : 2 * T::X * T::Y + 2 * T::X * (T::Z - 2) + 2 * (T::Y - 2) * (T::Z - 2);
}

// b-th face-layer vertex of a tile, in local coordinates (branch-free selects,
// so nothing is kept in private memory).
template <int NDIM>
__device__ __forceinline__ int3 face_vertex(int b) {
    using T = LabelTile<NDIM>;
    if constexpr (NDIM == 2) {
        const bool row = b < 2 * T::X;
        const int c = b - 2 * T::X;
        const int lx = row ? b % T::X : ((c / (T::Y - 2)) ? T::X - 1 : 0);
        const int ly = row ? ((b / T::X) ? T::Y - 1 : 0) : 1 + c % (T::Y - 2);
        return make_int3(lx, ly, 0);
    } else {
        constexpr int A = T::X * T::Y, Bn = T::X * (T::Z - 2);
        const int b1 = b - 2 * A, b2 = b1 - 2 * Bn;
        const int zf_x = b % T::X, zf_y = (b / T::X) % T::Y, zf_z = (b / A) ? T::Z - 1 : 0;
        const int yf_x = b1 % T::X, yf_z = 1 + (b1 / T::X) % (T::Z - 2), yf_y = (b1 / Bn) ? T::Y - 1 : 0;
        const int xf_y = 1 + b2 % (T::Y - 2), xf_z = 1 + (b2 / (T::Y - 2)) % (T::Z - 2);
        const int xf_x = (b2 / ((T::Y - 2) * (T::Z - 2))) ? T::X - 1 : 0;
        const bool zf = b < 2 * A, yf = !zf && b1 < 2 * Bn;
        return make_int3(zf ? zf_x : yf ? yf_x : xf_x, zf ? zf_y : yf ? yf_y : xf_y, zf ? zf_z : yf ? yf_z : xf_z);
    }
}

int label_tile_count(const Grid& gr) { return label_tiles_of(gr); }

// Origin of a label tile.
template <int NDIM>
__device__ __forceinline__ int3 tile_origin(const Grid& gr, int tile) {
    using T = LabelTile<NDIM>;
    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y;
    return make_int3((tile % tx_n) * T::X, ((tile / tx_n) % ty_n) * T::Y, (tile / (tx_n * ty_n)) * T::Z);
}

// The label tile of vertex i.
template <int NDIM>
__device__ __forceinline__ int tile_of_vertex(const Grid& gr, int i) {
    using T = LabelTile<NDIM>;
    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int x = i % gr.nx, y = (i / gr.nx) % gr.ny, z = NDIM == 3 ? i / gr.nxy : 0;
    return x / T::X + tx_n * (y / T::Y + ty_n * (z / T::Z));
}

// Pointer loads and stores of the compression walks.  Every value a walk can
// read is an ancestor of the vertex it came from (what the tile pass wrote, or
// a later shortcut on the same path), so the walks are correct whatever they
// see of each other's writes; workgroup scope keeps them cacheable in each
// XCD's L2 (the tile pass's results are there from the step before) instead
// of going to memory on every hop.
__device__ __forceinline__ int load_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void store_relaxed(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Walks qu[x] and qd[x] to the roots of x's two forests together (two
// independent chains, so their loads overlap), writing every step back.  The
// forests are acyclic (every pointer goes strictly up, resp. down, the total
// order), so the walks end; the step cap only guards against corrupted input
// and is reported as an error.
// acc counts the pointer loads and stores (4 bytes each).
constexpr int kMaxWalk = 1 << 22;
__device__ __forceinline__ bool compress_both(int* qu, int* qd, int x, int& ru, int& rd, unsigned& acc) {
    int yu = load_relaxed(qu + x), yd = load_relaxed(qd + x);
    acc += 2;
    for (int it = 0; it < kMaxWalk; ++it) {
        if (yu >= 0 && yd >= 0) {  // both roots
            ru = yu;
            rd = yd;
            return true;
        }
        const int zu = yu >= 0 ? yu : load_relaxed(qu - yu - 1);
        const int zd = yd >= 0 ? yd : load_relaxed(qd - yd - 1);
        acc += (yu < 0 ? 2u : 0u) + (yd < 0 ? 2u : 0u);
        if (yu < 0) store_relaxed(qu + x, zu), yu = zu;
        if (yd < 0) store_relaxed(qd + x, zd), yd = zd;
    }
    return false;
}

// Compresses the pointers of one tile's face-layer vertices to their roots
// (every exit target is one of them); false if a walk hit its cap.
// acc counts the 4-byte words the walks move.
template <int NDIM>
__device__ __forceinline__ bool compress_tile(const Grid& gr, int tile, int* __restrict__ q_up,
                                              int* __restrict__ q_dn, unsigned& acc) {
    constexpr int FC = face_count<NDIM>();
    const int3 o = tile_origin<NDIM>(gr, tile);
    bool ok = true;
    for (int b = threadIdx.x; b < FC; b += blockDim.x) {
        const int3 l = face_vertex<NDIM>(b);
        const int x = o.x + l.x, y = o.y + l.y, z = o.z + l.z;
        if (x >= gr.nx || y >= gr.ny || z >= gr.nz) continue;
        int ru, rd;
        ok = compress_both(q_up, q_dn, x + gr.nx * y + gr.nxy * z, ru, rd, acc) && ok;
    }
    return ok;
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_label_compress(Grid gr, int* __restrict__ q_up,
                                                        int* __restrict__ q_dn,
                                                        unsigned* __restrict__ cnt) {
    unsigned acc = 0;
    if (!compress_tile<NDIM>(gr, xcd_logical_block(blockIdx.x, gridDim.x), q_up, q_dn, acc))
        atomicOr(cnt + kCntErr, kErrWalk);
}

// Label-tile order: the gathers q[q[i]] of a tile land on the faces of the tile
// and its neighbours, so walking tiles (not rows) keeps them in cache.  A
// thread owns the 4-vertex row groups l = 4 t + 1024 k of its tile.
template <int NDIM>
struct TileGroup {
    int i0;     // global id of the group's first vertex
    int count;  // in-grid vertices of the group (0..4)
    bool vec;   // the four are in the grid, consecutive and 16-byte aligned
};

template <int NDIM>
__device__ __forceinline__ TileGroup<NDIM> tile_group(const Grid& gr, int tile, int k) {
    using T = LabelTile<NDIM>;
    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int bx = tile % tx_n, by = (tile / tx_n) % ty_n, bz = tile / (tx_n * ty_n);
    const int l0 = 4 * threadIdx.x + 1024 * k;
    const int xa = bx * T::X + l0 % T::X, y = by * T::Y + (l0 / T::X) % T::Y, z = bz * T::Z + l0 / (T::X * T::Y);
    TileGroup<NDIM> g;
    g.i0 = xa + gr.nx * y + gr.nxy * z;
    g.count = (y < gr.ny && z < gr.nz) ? max(0, min(4, gr.nx - xa)) : 0;
    g.vec = g.count == 4 && (gr.nx & 3) == 0;
    return g;
}

// Writes the final labels (the root at the end of each vertex's chain), tile
// by tile; returns kErrWalk if a chain hit the step cap.  May run in place
// (M == q_up, m == q_dn): a value read is then a pointer along the chain or,
// once written, its root.
template <int NDIM>
__device__ __forceinline__ unsigned label_final_tile(const int* q_up, const int* q_dn, const Grid& gr, int tile,
                                                     int* M, int* m, unsigned& hops) {
    constexpr int G = LabelTile<NDIM>::X * LabelTile<NDIM>::Y * LabelTile<NDIM>::Z / 1024;
    int a[G][4], b[G][4];
    TileGroup<NDIM> tg[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        tg[k] = tile_group<NDIM>(gr, tile, k);
#pragma unroll
        for (int j = 0; j < 4; ++j) a[k][j] = b[k][j] = 0;
        if (tg[k].vec) {
            const int4 u = *reinterpret_cast<const int4*>(q_up + tg[k].i0);
            const int4 d = *reinterpret_cast<const int4*>(q_dn + tg[k].i0);
            a[k][0] = u.x, a[k][1] = u.y, a[k][2] = u.z, a[k][3] = u.w;
            b[k][0] = d.x, b[k][1] = d.y, b[k][2] = d.z, b[k][3] = d.w;
        } else {
            for (int j = 0; j < tg[k].count; ++j) a[k][j] = q_up[tg[k].i0 + j], b[k][j] = q_dn[tg[k].i0 + j];
        }
    }
    unsigned bad = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        int y[8];  // a group's up and down chains, walked together
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            y[2 * j] = j < tg[k].count ? a[k][j] : 0;
            y[2 * j + 1] = j < tg[k].count ? b[k][j] : 0;
        }
        follow_roots<8>(q_up, q_dn, y, bad, hops);
        int ra[4], rb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ra[j] = y[2 * j];
            rb[j] = y[2 * j + 1];
        }
        if (tg[k].vec) {
            *reinterpret_cast<int4*>(M + tg[k].i0) = make_int4(ra[0], ra[1], ra[2], ra[3]);
            *reinterpret_cast<int4*>(m + tg[k].i0) = make_int4(rb[0], rb[1], rb[2], rb[3]);
        } else {
            for (int j = 0; j < tg[k].count; ++j) M[tg[k].i0 + j] = ra[j], m[tg[k].i0 + j] = rb[j];
        }
    }
    return bad;
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_label_final(const int* q_up, const int* q_dn, Grid gr, int* M,
                                                     int* m, unsigned* __restrict__ cnt) {
    const ItemRange range = xcd_items(label_tiles_of(gr));
    unsigned bad = 0, hops = 0;
    for (int tile = range.first; tile < range.hi; tile += range.stride)
        bad |= label_final_tile<NDIM>(q_up, q_dn, gr, tile, M, m, hops);
    if (bad) atomicOr(cnt + kCntErr, bad);
}

// LDS of a step kernel: two flag-gather lists of kEngChunk vertices, the
// stencil planes, or the troublemakers' targets.
constexpr int kEngSmemBytes = 2 * kEngChunk * sizeof(int);

// The troublemakers' targets found by one block, kept in LDS until its tiles
// are done; a target beyond the list's capacity is edited at once.
struct TargetList {
    static constexpr int kCap = kEngSmemBytes / 2 / sizeof(int);  // the other half: the candidate lists
    int* list;  // nullptr: count only
    unsigned* count;
    uint8_t* marks;
    float* g;
    const float* L;
    Dirty dirty;
    bool preempt;  // edits without claims (preemptive mode)
    template <int NDIM>
    __device__ __forceinline__ void put(const Grid& gr, unsigned k, int t, unsigned& changed) const {
        if (k < static_cast<unsigned>(kCap)) list[k] = t;
        else target_edit<NDIM>(preempt, marks, g, L, dirty, gr, t, changed);
    }
    // Appends each lane's targets (-1: none; nloc of them): one LDS atomic per
    // wave, positions from a prefix sum over the wave.
    template <int NDIM>
    __device__ __forceinline__ void add_wave(const Grid& gr, const int (&tn)[4], const int (&tx)[4], int nloc,
                                             unsigned& changed) const {
        if (!__any(nloc)) return;
        const int lane = threadIdx.x & 63;
        int incl = nloc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        unsigned base = 0;
        if (lane == 63) base = atomicAdd(count, static_cast<unsigned>(incl));
        unsigned k = __shfl(base, 63) + static_cast<unsigned>(incl - nloc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (tn[j] >= 0) put<NDIM>(gr, k++, tn[j], changed);
            if (tx[j] >= 0) put<NDIM>(gr, k++, tx[j], changed);
        }
    }
};

// Troublemakers of one tile (Sec. 5.2).  Only a vertex whose direction in g
// differs from f's (each family apart) can be one, so only such vertices
// have their labels resolved -- their pointers in g's and f's forests (Mf,
// mf hold f's tile pointers) loaded and both exit chains followed; the rest
// of the tile costs its two direction bytes per vertex.  Mislabelled vertices need not be counted for the loop:
// one exists exactly when a troublemaker of its family does (on the steepest
// path in g of a mislabelled vertex, the first vertex whose direction
// differs from f's carries the same labels in g and in f), so the
// troublemaker count ends the R loop alike.  With full set, every vertex's
// labels are resolved and the mislabelled ones counted in wrong (the start
// field's count; the loop's rounds use detect_r_tile_sparse, below).  bytes
// receives the algorithmic bytes of the loads.
template <int NDIM>
__device__ __forceinline__ void detect_r_tile(const uint8_t* __restrict__ dirs_f, const uint8_t* __restrict__ dirs_g,
                                              const int* __restrict__ q_up, const int* __restrict__ q_dn,
                                              const int* __restrict__ Mf, const int* __restrict__ mf, const Grid& gr,
                                              int tile, bool full, bool flabels, const TargetList& tl, unsigned& wrong,
                                              unsigned& cases, unsigned& changed, unsigned& bad, unsigned& hops,
                                              unsigned long long& bytes) {
    constexpr int G = LabelTile<NDIM>::X * LabelTile<NDIM>::Y * LabelTile<NDIM>::Z / 1024;
    static_assert(G == 4, "four row groups per thread");
    // every direction word of the tile first, all in flight together (kept
    // in named registers: the group loop below is not unrolled, and an array
    // indexed by its counter would go to private memory)
    unsigned w[2 * G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const TileGroup<NDIM> t = tile_group<NDIM>(gr, tile, k);
        unsigned a = 0u, b = 0u;
        if (t.vec) {
            a = *reinterpret_cast<const unsigned*>(dirs_f + t.i0);
            b = *reinterpret_cast<const unsigned*>(dirs_g + t.i0);
        } else {
            for (int j = 0; j < t.count; ++j) {
                a |= static_cast<unsigned>(dirs_f[t.i0 + j]) << (8 * j);
                b |= static_cast<unsigned>(dirs_g[t.i0 + j]) << (8 * j);
            }
        }
        w[2 * k] = a;
        w[2 * k + 1] = b;
    }
    const unsigned f0 = w[0], g0 = w[1], f1 = w[2], g1 = w[3], f2 = w[4], g2 = w[5], f3 = w[6], g3 = w[7];
#pragma unroll 1
    for (int k = 0; k < G; ++k) {
        const unsigned dfw = k == 0 ? f0 : k == 1 ? f1 : k == 2 ? f2 : f3;
        const unsigned dgw = k == 0 ? g0 : k == 1 ? g1 : k == 2 ? g2 : g3;
        // bit j: vertex j's ascent (dup) / descent (ddn) differs (bytes past
        // the group's count are equal zeros); up, dn: the labels to resolve
        const unsigned x = dfw ^ dgw;
        unsigned dup = 0, ddn = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dup |= ((x >> (8 * j + 4)) & 15u) ? 1u << j : 0u;
            ddn |= ((x >> (8 * j)) & 15u) ? 1u << j : 0u;
        }
        const TileGroup<NDIM> t = tile_group<NDIM>(gr, tile, k);
        const unsigned all = (1u << t.count) - 1u;
        const unsigned up = full ? all : dup, dn = full ? all : ddn;
        if (!__any(up | dn)) continue;
        const int i0 = t.i0;
        // pointers and f's labels of the differing vertices (int4 lanes x..w
        // are the group's vertices 0..3; no arrays, which would be indexed
        // at run time in the scalar path and go to private memory)
        int4 u = make_int4(0, 0, 0, 0), U = u, d = u, D = u;
        if (t.vec) {
            if (up) {
                u = *reinterpret_cast<const int4*>(q_up + i0);
                U = *reinterpret_cast<const int4*>(Mf + i0);
                bytes += 32;
            }
            if (dn) {
                d = *reinterpret_cast<const int4*>(q_dn + i0);
                D = *reinterpret_cast<const int4*>(mf + i0);
                bytes += 32;
            }
        } else {  // bits past the count are clear
            if (up & 1u) u.x = q_up[i0], U.x = Mf[i0];
            if (up & 2u) u.y = q_up[i0 + 1], U.y = Mf[i0 + 1];
            if (up & 4u) u.z = q_up[i0 + 2], U.z = Mf[i0 + 2];
            if (up & 8u) u.w = q_up[i0 + 3], U.w = Mf[i0 + 3];
            if (dn & 1u) d.x = q_dn[i0], D.x = mf[i0];
            if (dn & 2u) d.y = q_dn[i0 + 1], D.y = mf[i0 + 1];
            if (dn & 4u) d.z = q_dn[i0 + 2], D.z = mf[i0 + 2];
            if (dn & 8u) d.w = q_dn[i0 + 3], D.w = mf[i0 + 3];
            bytes += 8 * (__popc(up) + __popc(dn));
        }
        // chains of the differing directions only (0: nothing to follow) in
        // g's forest, then f's labels along f's chains (entries 8..15): with
        // f's labels resolved (flabels) they are roots already; else both
        // forests' chains are followed in the same passes
        int y[16] = {(up & 1u) ? u.x : 0, (dn & 1u) ? d.x : 0, (up & 2u) ? u.y : 0, (dn & 2u) ? d.y : 0,
                     (up & 4u) ? u.z : 0, (dn & 4u) ? d.z : 0, (up & 8u) ? u.w : 0, (dn & 8u) ? d.w : 0,
                     (up & 1u) ? U.x : 0, (dn & 1u) ? D.x : 0, (up & 2u) ? U.y : 0, (dn & 2u) ? D.y : 0,
                     (up & 4u) ? U.z : 0, (dn & 4u) ? D.z : 0, (up & 8u) ? U.w : 0, (dn & 8u) ? D.w : 0};
        if (flabels) {
            int yg[8] = {y[0], y[1], y[2], y[3], y[4], y[5], y[6], y[7]};
            int yf[8] = {y[8], y[9], y[10], y[11], y[12], y[13], y[14], y[15]};
            follow_roots<8>(q_up, q_dn, yg, bad, hops);
            follow_roots<8>(Mf, mf, yf, bad, hops);
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = yg[k], y[8 + k] = yf[k];
        } else {
            follow_roots<16, 8>(q_up, q_dn, y, bad, hops, Mf, mf);
        }
        const int Ms[4] = {y[8], y[10], y[12], y[14]}, ms[4] = {y[9], y[11], y[13], y[15]};
        int tn[4], tx[4], nloc = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            tn[j] = tx[j] = -1;
            const int i = i0 + j;
            const unsigned df = (dfw >> (8 * j)) & 0xFFu, dg = (dgw >> (8 * j)) & 0xFFu;
            const bool wM = ((up >> j) & 1u) && y[2 * j] != Ms[j];
            const bool wm = ((dn >> j) & 1u) && y[2 * j + 1] != ms[j];
            wrong += wM || wm;  // all resolved only when full
            const bool rmax = wM && ((dup >> j) & 1u);
            const bool rmin = wm && ((ddn >> j) & 1u);
            cases += rmin + rmax;
            nloc += rmin + rmax;
            if (rmin) tn[j] = i + slot_offset(gr, df & 15u);
            if (rmax) tx[j] = i + slot_offset(gr, dg >> 4);
        }
        if (tl.list) tl.add_wave<NDIM>(gr, tn, tx, nloc, changed);
    }
}

// Global id of the vertex with tile-local index l (l = x + X (y + Y z) in the
// tile's box).
template <int NDIM>
__device__ __forceinline__ int tile_vertex(const Grid& gr, int tile, int l) {
    using T = LabelTile<NDIM>;
    const int tx_n = (gr.nx + T::X - 1) / T::X, ty_n = (gr.ny + T::Y - 1) / T::Y;
    const int bx = tile % tx_n, by = (tile / tx_n) % ty_n, bz = tile / (tx_n * ty_n);
    const int x = bx * T::X + l % T::X, y = by * T::Y + (l / T::X) % T::Y, z = bz * T::Z + l / (T::X * T::Y);
    return x + gr.nx * y + gr.nxy * z;
}

// The troublemakers of one tile as detect_r_tile finds them without full, in
// two phases: the vertices whose ascent (descent) differs are listed in LDS
// first (cand_up / cand_dn, 4096 entries each: the tile-local index in bits
// 0..11 and the slot of the target's direction -- g's ascent, f's descent --
// in bits 12..15; *s_n counts them, ascents in its low and descents in its
// high 16 bits, and is 0 on entry and on return), then resolved four per
// thread, every walk of a round in flight together.  A wave then waits for
// one round of pointer loads and walks per 1024 listed vertices of the tile
// instead of one per row group it holds.
template <int NDIM>
__device__ __forceinline__ void detect_r_tile_sparse(const uint8_t* __restrict__ dirs_f,
                                                     const uint8_t* __restrict__ dirs_g,
                                                     const int* __restrict__ q_up, const int* __restrict__ q_dn,
                                                     const int* __restrict__ Mf, const int* __restrict__ mf,
                                                     const Grid& gr, int tile, const TargetList& tl,
                                                     unsigned short* cand_up, unsigned short* cand_dn, unsigned* s_n,
                                                     unsigned& cases, unsigned& changed, unsigned& bad,
                                                     unsigned& hops, unsigned long long& bytes) {
    using T = LabelTile<NDIM>;
    constexpr int G = T::X * T::Y * T::Z / 1024;
    static_assert(G == 4 && T::X * T::Y * T::Z == 4096, "4096 vertices, four row groups per thread");
    unsigned w[2 * G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const TileGroup<NDIM> t = tile_group<NDIM>(gr, tile, k);
        unsigned a = 0u, b = 0u;
        if (t.vec) {
            a = *reinterpret_cast<const unsigned*>(dirs_f + t.i0);
            b = *reinterpret_cast<const unsigned*>(dirs_g + t.i0);
        } else {  // bytes past the count stay equal zeros
            for (int j = 0; j < t.count; ++j) {
                a |= static_cast<unsigned>(dirs_f[t.i0 + j]) << (8 * j);
                b |= static_cast<unsigned>(dirs_g[t.i0 + j]) << (8 * j);
            }
        }
        w[2 * k] = a;
        w[2 * k + 1] = b;
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const unsigned dfw = w[2 * k], dgw = w[2 * k + 1], x = dfw ^ dgw;
        unsigned dup = 0, ddn = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dup |= ((x >> (8 * j + 4)) & 15u) ? 1u << j : 0u;
            ddn |= ((x >> (8 * j)) & 15u) ? 1u << j : 0u;
        }
        if (!__any(dup | ddn)) continue;
        const unsigned mine = static_cast<unsigned>(__popc(dup)) | (static_cast<unsigned>(__popc(ddn)) << 16);
        unsigned incl = mine;  // each half stays below 2^13: no carry between them
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        unsigned base = 0;
        if (lane == 63) base = atomicAdd(s_n, incl);
        base = __shfl(base, 63);
        const unsigned before = incl - mine;
        unsigned pu = (base & 0xFFFFu) + (before & 0xFFFFu), pd = (base >> 16) + (before >> 16);
        const unsigned l0 = 4u * threadIdx.x + 1024u * k;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if ((dup >> j) & 1u) cand_up[pu++] = static_cast<unsigned short>((l0 + j) | (((dgw >> (8 * j + 4)) & 15u) << 12));
            if ((ddn >> j) & 1u) cand_dn[pd++] = static_cast<unsigned short>((l0 + j) | (((dfw >> (8 * j)) & 15u) << 12));
        }
    }
    __syncthreads();
    const unsigned nn = *s_n;
    const int nu = static_cast<int>(nn & 0xFFFFu), n = nu + static_cast<int>(nn >> 16);
    for (int b0 = 0; b0 < n; b0 += 4 * static_cast<int>(blockDim.x)) {  // block-uniform rounds
        int vi[4], yg[4], yf[4];
        unsigned code[4];
        bool dn[4], ok[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = b0 + e * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
            ok[e] = idx < n;
            dn[e] = idx >= nu;
            code[e] = ok[e] ? (dn[e] ? cand_dn[idx - nu] : cand_up[idx]) : 0u;
            vi[e] = ok[e] ? tile_vertex<NDIM>(gr, tile, static_cast<int>(code[e] & 4095u)) : 0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // g's tile pointer and f's (a label when f's are resolved)
            yg[e] = ok[e] ? (dn[e] ? q_dn : q_up)[vi[e]] : 0;
            yf[e] = ok[e] ? (dn[e] ? mf : Mf)[vi[e]] : 0;
        }
        // both walks of every entry, one gather level per pass
        for (int pass = 0;; ++pass) {
            bool any = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) any |= (yg[e] < 0) | (yf[e] < 0);
            if (!any) break;
            if (pass == kMaxChain) {
                bad = kErrWalk;
#pragma unroll
                for (int e = 0; e < 4; ++e) yg[e] = max(yg[e], 0), yf[e] = max(yf[e], 0);
                break;
            }
            int zg[4], zf[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                zg[e] = (dn[e] ? q_dn : q_up)[yg[e] < 0 ? -yg[e] - 1 : 0];
                zf[e] = (dn[e] ? mf : Mf)[yf[e] < 0 ? -yf[e] - 1 : 0];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                hops += (yg[e] < 0) + (yf[e] < 0);
                yg[e] = yg[e] < 0 ? zg[e] : yg[e];
                yf[e] = yf[e] < 0 ? zf[e] : yf[e];
            }
        }
        // a listed vertex with different labels is a troublemaker; its target
        // is the neighbour along g's ascent (max) or f's descent (min)
        int tn[4], tx[4], nloc = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            tn[e] = tx[e] = -1;
            bytes += ok[e] ? 8u : 0u;
            if (ok[e] && yg[e] != yf[e]) {
                const int t = vi[e] + slot_offset(gr, code[e] >> 12);
                if (dn[e]) tn[e] = t;
                else tx[e] = t;
                ++cases;
                ++nloc;
            }
        }
        if (tl.list) tl.add_wave<NDIM>(gr, tn, tx, nloc, changed);
    }
    __syncthreads();  // every entry read before the next tile lists its own
    if (threadIdx.x == 0) *s_n = 0u;
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
    unsigned bad = 0, hops = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned bits = case_bits(dirs_f[i], dirs_g[i]);
        c[0] += bits & 1u;
        c[1] += (bits >> 1) & 1u;
        c[2] += (bits >> 2) & 1u;
        c[3] += (bits >> 3) & 1u;
        int yg[2] = {qgu[i], qgd[i]}, yf[2] = {qfu[i], qfd[i]};
        follow_roots<2>(qgu, qgd, yg, bad, hops);
        follow_roots<2>(qfu, qfd, yf, bad, hops);
        const bool wM = yg[0] != yf[0];
        const bool wm = yg[1] != yf[1];
        c[4] += wM;
        c[5] += wm;
        c[6] += wM || wm;
    }
    const int idx[7] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3,
                        kCntWrongMax, kCntWrongMin, kCntWrong};
    if (bad) atomicOr(cnt + kCntErr, bad);
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

// Deltas of the 4-vertex group w (vector path when the group is whole).
__device__ __forceinline__ void delta_group(const float* __restrict__ g, const float* __restrict__ fhat, int n,
                                            float* __restrict__ delta, float* __restrict__ g_out, int w,
                                            unsigned& edited, unsigned& inexact) {
    if (4 * w + 3 < n) {
        const float4 g4 = reinterpret_cast<const float4*>(g)[w];
        const float4 h4 = reinterpret_cast<const float4*>(fhat)[w];
        const float4 d4 = make_float4(delta_one(g4.x, h4.x, edited, inexact), delta_one(g4.y, h4.y, edited, inexact),
                                      delta_one(g4.z, h4.z, edited, inexact), delta_one(g4.w, h4.w, edited, inexact));
        reinterpret_cast<float4*>(delta)[w] = d4;
        if (g_out) reinterpret_cast<float4*>(g_out)[w] = g4;
    } else {
        for (int i = 4 * w; i < n; ++i) {
            const float gi = g[i];
            delta[i] = delta_one(gi, fhat[i], edited, inexact);
            if (g_out) g_out[i] = gi;
        }
    }
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
// Tile variants of the direction kernel selectable per call (index 1..);
// index 0 is the default (2D: 64 x 16 tiles; 3D: 64 x 16 x 16 columns).
__host__ __device__ inline DirsVariant variant_of(int ndim, int v) {
    if (ndim == 2) return v == 2 ? DirsVariant{32, 1} : DirsVariant{16, 1};
    switch (v) {
        case 2: return {16, 8};
        case 3: return {16, 32};
        case 4: return {32, 16};
        default: return {16, 16};
    }
}

int tile_variant_count(int ndim) { return ndim == 2 ? 2 : 4; }

// Persistent grid: at most kDirsBlocks blocks (8 per compute unit), each walking
// a contiguous run of work items of its XCD.
constexpr int kDirsBlocks = 2048;

template <int NDIM, int TY, int ZC>
static void launch_dirs_t(const float* h, const Grid& gr, uint8_t* dirs_out, hipStream_t s) {
    const int tx = (gr.nx + kTileX - 1) / kTileX;
    const int ty = (gr.ny + TY - 1) / TY;
    const int tz = NDIM == 3 ? (gr.nz + ZC - 1) / ZC : 1;
    const int items = tx * ty * tz;
    const int nb = items < kDirsBlocks ? items : kDirsBlocks;
    hipLaunchKernelGGL((k_dirs<NDIM, TY, ZC>), dim3(nb), dim3(256), 0, s, h, gr, dirs_out);
}

void launch_dirs(const float* h, const Grid& gr, int variant, uint8_t* dirs_out, hipStream_t s) {
    if (gr.ndim == 2) {
        if (variant_of(2, variant).ty == 32) launch_dirs_t<2, 32, 1>(h, gr, dirs_out, s);
        else launch_dirs_t<2, 16, 1>(h, gr, dirs_out, s);
    } else {
        const DirsVariant v = variant_of(3, variant);
        if (v.ty == 32) launch_dirs_t<3, 32, 16>(h, gr, dirs_out, s);
        else if (v.zc == 8) launch_dirs_t<3, 16, 8>(h, gr, dirs_out, s);
        else if (v.zc == 32) launch_dirs_t<3, 16, 32>(h, gr, dirs_out, s);
        else launch_dirs_t<3, 16, 16>(h, gr, dirs_out, s);
    }
}

void launch_label_tile(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, hipStream_t s) {
    const int nb = label_tiles_of(gr);
    if (gr.ndim == 2) hipLaunchKernelGGL(k_label_tile<2>, dim3(nb), dim3(256), 0, s, dirs, gr, q_up, q_dn);
    else hipLaunchKernelGGL(k_label_tile<3>, dim3(nb), dim3(256), 0, s, dirs, gr, q_up, q_dn);
}

void launch_label_compress(const Grid& gr, int* q_up, int* q_dn, unsigned* cnt, hipStream_t s) {
    const int nb = label_tiles_of(gr);
    if (gr.ndim == 2) hipLaunchKernelGGL(k_label_compress<2>, dim3(nb), dim3(256), 0, s, gr, q_up, q_dn, cnt);
    else hipLaunchKernelGGL(k_label_compress<3>, dim3(nb), dim3(256), 0, s, gr, q_up, q_dn, cnt);
}

void launch_label_forests(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, unsigned* cnt,
                          hipStream_t s) {
    launch_label_tile(dirs, gr, q_up, q_dn, s);
    launch_label_compress(gr, q_up, q_dn, cnt, s);
}

void launch_label_final(const int* q_up, const int* q_dn, const Grid& gr, int* M, int* m, unsigned* cnt,
                        hipStream_t s) {
    const int nt = label_tiles_of(gr);
    const int nb = nt < kDirsBlocks ? nt : kDirsBlocks;
    if (gr.ndim == 2) hipLaunchKernelGGL(k_label_final<2>, dim3(nb), dim3(256), 0, s, q_up, q_dn, gr, M, m, cnt);
    else hipLaunchKernelGGL(k_label_final<3>, dim3(nb), dim3(256), 0, s, q_up, q_dn, gr, M, m, cnt);
}

void launch_compare(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* qfu, const int* qfd,
                    const int* qgu, const int* qgd, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_compare, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, dirs_f, dirs_g,
                       qfu, qfd, qgu, qgd, n, cnt);
}

void launch_check_finite(const float* h, int n, unsigned* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(n, 256 * 4, kGridCap)), dim3(256), 0, s, h, n, cnt);
}

// ============================================================ batch engine ==
//
// The schedule of the correction loop (Sec. 5) runs on the device.  A step
// advances every unfinished field of a batch by one operation of its own
// schedule -- the same sequence of operations for every field as for a field
// corrected alone, so results are identical.  One field: k_eng_step1 decides
// in every block and runs the chosen operation, one kernel per step.  A
// batch: k_eng_step<NDIM> runs the work items of all fields of one dimension
// as one index space, cut into contiguous ranges per block (XCD-aware, so
// neighbouring items share an L2), and its last blocks reduce each field's
// counters, write its next operation and split the next step's items over
// the blocks.  The host captures a fixed number of steps in a HIP graph and
// relaunches it until no field is active; a batch's 2D fields and 3D fields
// form two chains of steps, each with its own graph.  Kernel boundaries order
// the steps: every write of a step is visible to the next one without
// device-scope fences inside a kernel (which on MI355X write back and
// invalidate the L2 of each XCD).

__host__ __device__ inline int dirs_items_of(const Grid& gr, int variant) {
    const DirsVariant v = variant_of(gr.ndim, variant);
    const int tx = (gr.nx + kTileX - 1) / kTileX, ty = (gr.ny + v.ty - 1) / v.ty;
    const int tz = gr.ndim == 3 ? (gr.nz + v.zc - 1) / v.zc : 1;
    return tx * ty * tz;
}

__host__ __device__ inline int eng_items(const EngField& F, int op) {
    const int chunks = (F.gr.n + kEngChunk - 1) / kEngChunk;
    const int tiles = label_tiles_of(F.gr);
    const int dirs = dirs_items_of(F.gr, F.variant);
    switch (op) {
        case kOpPreA: case kOpApplyC: case kOpRefreshC: case kOpRefreshR: case kOpDelta:
            return chunks;
        case kOpPreB: case kOpPreD: case kOpRTile: case kOpRDetect: return tiles;
        case kOpPreA2: case kOpPreE: case kOpFullC: case kOpFullR: return dirs;
        default: return 0;
    }
}

int eng_items_host(const EngField& F, int op) { return eng_items(F, op); }

// Cost of one work item of op, in units of about 1 us of one block (per-item
// block times measured inside the 96-field batch): a batch step splits the
// weighted index space, not the item count, evenly over its blocks, so a
// block that draws troublemaker tiles draws fewer of them than one that
// draws sparse apply chunks.  Direction items scale with their tile's vertex
// count (per 4096 vertices: 5.6 for the directions of f, 8.5 with the cases).
__host__ __device__ inline int eng_weight(const EngField& F, int op) {
    const DirsVariant v = variant_of(F.gr.ndim, F.variant);
    const int dv = kTileX * v.ty * (F.gr.ndim == 3 ? v.zc : 1);  // vertices of a direction item
    switch (op) {
        case kOpPreA: return F.warm ? 12 : 10;
        case kOpPreA2: return (56 * dv + 10 * kEngChunk - 1) / (10 * kEngChunk);
        case kOpPreE: case kOpFullC: case kOpFullR: return (85 * dv + 10 * kEngChunk - 1) / (10 * kEngChunk);
        case kOpPreB: return 21;
        case kOpPreD: return 22;
        case kOpRTile: return 13;  // the clean tiles of g are skipped
        case kOpRDetect: return 22;
        case kOpApplyC: case kOpRefreshC: return 2;
        case kOpRefreshR: return 3;
        case kOpDelta: return 5;
        default: return 1;
    }
}

int eng_weight_host(const EngField& F, int op) { return eng_weight(F, op); }

// Direction work items [a, b) of field F with its variant's tile shape.
template <int NDIM, int MODE>
__device__ __forceinline__ void eng_dirs(const EngField& F, const float* h, uint8_t* out, int a, int b, float* sm,
                                         unsigned (&c)[4]) {
    const ItemRange r{a, b, 1};
    const Grid& gr = F.gr;
    const CaseArrays ca{F.cases, F.dirty, F.marks};
    if constexpr (NDIM == 2) {
        if (variant_of(2, F.variant).ty == 32) dirs_stream<2, 32, 1, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
        else dirs_stream<2, 16, 1, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
    } else {
        const DirsVariant v = variant_of(3, F.variant);
        if (v.ty == 32) dirs_stream<3, 32, 16, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
        else if (v.zc == 8) dirs_stream<3, 16, 8, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
        else if (v.zc == 32) dirs_stream<3, 16, 32, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
        else dirs_stream<3, 16, 16, MODE>(h, gr, r, out, F.dirs_f, ca, sm, c);
    }
}

// Steepest ascent and descent of vertex i in g, read straight from memory
// (the refresh of a few vertices): the same neighbour order and comparisons
// as the stencil (odd slots have the smaller ids, even slots the larger ones,
// each nearest first), with neighbours outside the grid left out.
template <int NDIM>
__device__ __forceinline__ unsigned steepest_at(const float* __restrict__ g, const Grid& gr, int i) {
    constexpr int NS = NDIM == 3 ? 14 : 6;
    const int x = i % gr.nx, y = (i / gr.nx) % gr.ny, z = NDIM == 3 ? i / gr.nxy : 0;
    const float nan = __builtin_nanf("");
    float w[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) w[s] = slot_in_grid<NDIM>(gr, x, y, z, s) ? g[i + gr.off[s]] : nan;
    const float v = g[i];
    Steepest b{v, v, kSelf, kSelf};
#pragma unroll
    for (int s = 1; s < NS; s += 2) b.below(w[s], s);
#pragma unroll
    for (int s = 0; s < NS; s += 2) b.above(w[s], s);
    return (b.us << 4) | b.ds;
}

// Runs fn(v) for every flagged vertex v of the chunks [lo, hi) (kEngChunk
// vertices each; thread t loads the 16 flag bytes t of a chunk, and a byte
// flags its vertex when it has a bit of `mask` set; bytes past the grid are
// never set).  With use_sel, a range of at least kSelectChunks chunks reads only the
// chunks c with sel(c): the block evaluates sel for 256 chunks at once (one
// per thread) and takes the selected ones from its ballots, so a range with
// none costs one summary load per thread; after chunk c was read, thread 0
// calls done(c, w0, w1), where with COUNT w0 and w1 hold the numbers of its
// bytes with bit 0 and 1 (low and high 16 bits of w0) and bit 2 and 3 (w1)
// set.  A shorter range reads every chunk and calls neither (its summaries
// are left as they were).  The flagged vertices are gathered into an LDS
// list so that all threads of the block work on them at once: one memory
// round trip for the whole range instead of one per vertex and thread.
// after_load(w) runs once per loaded word w that flagged something, after
// it was read.  list: LDS of kEngChunk ints; wsum: 4 ints.  Returns the
// number of chunks read.
template <bool COUNT, typename Sel, typename Done, typename Fn, typename AfterLoad>
__device__ __forceinline__ int for_flagged(const uint8_t* flags, int n, int lo, int hi, unsigned mask, bool use_sel,
                                           int* list, int* wsum, Sel&& sel, Done&& done, Fn&& fn,
                                           AfterLoad&& after_load) {
    constexpr int MAXW = 4;  // chunks gathered together
    const int nw = (n + 15) >> 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool select = use_sel && hi - lo >= kSelectChunks;  // block-uniform
    __shared__ unsigned long long s_sel[4];
    __shared__ unsigned s_cnt[MAXW][2];
    if (COUNT && select && threadIdx.x < 2 * MAXW) s_cnt[threadIdx.x >> 1][threadIdx.x & 1] = 0u;  // read after a barrier
    int read = 0;
    // one group of up to MAXW chunks (-1: none)
    auto group = [&](const int (&ch)[MAXW]) {
        unsigned m[MAXW][4];
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            read += ch[k] >= 0;
            const int w = ch[k] * (kEngChunk / 16) + threadIdx.x;
            const uint4 u = (ch[k] >= 0 && w < nw) ? reinterpret_cast<const uint4*>(flags)[w]
                                                   : make_uint4(0u, 0u, 0u, 0u);
            if (COUNT && select) {  // bytes with bit t set, over the block (16-bit lanes: at most 4096)
                unsigned c01 = 0u, c23 = 0u;
                const unsigned q4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    c01 += __popc(q4[q] & 0x01010101u) + 65536u * __popc(q4[q] & 0x02020202u);
                    c23 += __popc(q4[q] & 0x04040404u) + 65536u * __popc(q4[q] & 0x08080808u);
                }
#pragma unroll
                for (int sh = 32; sh > 0; sh >>= 1) {
                    c01 += __shfl_xor(c01, sh);
                    c23 += __shfl_xor(c23, sh);
                }
                if (lane == 0 && ch[k] >= 0) {
                    atomicAdd(&s_cnt[k][0], c01);
                    atomicAdd(&s_cnt[k][1], c23);
                }
            }
            m[k][0] = u.x & mask, m[k][1] = u.y & mask, m[k][2] = u.z & mask, m[k][3] = u.w & mask;
        }
#pragma unroll
        for (int k = 0; k < MAXW; ++k) {
            const unsigned any = m[k][0] | m[k][1] | m[k][2] | m[k][3];
            if (any) after_load(ch[k] * (kEngChunk / 16) + threadIdx.x);
            // one flagged vertex per byte: count the bytes with a bit set
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned b = m[k][q];
                const unsigned nz =
                    (b | (b >> 1) | (b >> 2) | (b >> 3) | (b >> 4) | (b >> 5) | (b >> 6) | (b >> 7)) & 0x01010101u;
                m[k][q] = nz;
                cnt += __popc(nz);
            }
        }
        // exclusive prefix of cnt over the block
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();  // wsum and s_cnt are complete
        int base_pos = 0, total = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = wsum[k];
            base_pos += k < wave ? t : 0;
            total += t;
        }
        if (select && threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < MAXW; ++k)
                if (ch[k] >= 0) {
                    done(ch[k], COUNT ? s_cnt[k][0] : 0u, COUNT ? s_cnt[k][1] : 0u);
                    if (COUNT) s_cnt[k][0] = s_cnt[k][1] = 0u;
                }
        }
        __syncthreads();  // wsum and s_cnt are rewritten by the next group
        // the list holds kEngChunk entries; more are done in several passes
        for (int pass = 0; pass * kEngChunk < total; ++pass) {
            const int p0 = pass * kEngChunk;
            int pos = base_pos + incl - cnt;
            if (pos < p0 + kEngChunk && pos + cnt > p0) {
#pragma unroll
                for (int k = 0; k < MAXW; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        unsigned bb = m[k][q];
                        while (bb) {
                            const int b = (__ffs(bb) - 1) >> 3;
                            bb &= bb - 1u;
                            if (pos >= p0 && pos < p0 + kEngChunk)
                                list[pos - p0] = ch[k] * kEngChunk + 16 * threadIdx.x + 4 * q + b;
                            ++pos;
                        }
                    }
            }
            __syncthreads();
            const int np = min(kEngChunk, total - p0);
            for (int e = threadIdx.x; e < np; e += blockDim.x) fn(list[e]);
            __syncthreads();  // the list is rewritten next
        }
    };
    if (!select) {
        for (int c0 = lo; c0 < hi; c0 += MAXW) {
            int ch[MAXW];
#pragma unroll
            for (int k = 0; k < MAXW; ++k) ch[k] = c0 + k < hi ? c0 + k : -1;
            group(ch);
        }
        return read;
    }
    for (int base = lo; base < hi; base += 256) {
        const int mine = base + static_cast<int>(threadIdx.x);
        const unsigned long long bw = __ballot(mine < hi && sel(mine));
        if (lane == 0) s_sel[wave] = bw;
        __syncthreads();
        unsigned long long sel4[4];  // block-uniform
#pragma unroll
        for (int w = 0; w < 4; ++w) sel4[w] = s_sel[w];
        __syncthreads();  // s_sel is rewritten by the next window
        for (int sw = 0; sw < 4; ++sw) {
            unsigned long long bits = sel4[sw];
            while (bits) {
                int ch[MAXW];
#pragma unroll
                for (int k = 0; k < MAXW; ++k) {
                    ch[k] = bits ? base + 64 * sw + __ffsll(static_cast<long long>(bits)) - 1 : -1;
                    bits &= bits - 1;
                }
                group(ch);
            }
        }
    }
    return read;
}

__device__ __forceinline__ Dirty dirty_of(const EngField& F, bool sum) { return Dirty{F.dirty, sum ? F.chunk_dirty : nullptr}; }

// An apply's record of a chunk it read in full: its exact case counts.
__device__ __forceinline__ auto chunk_counted(const EngField& F) {
    return [&F](int c, unsigned w0, unsigned w1) {
        F.chunk_cnt[2 * c] = w0;
        F.chunk_cnt[2 * c + 1] = w1;
        F.chunk_unk[c] = 0u;
    };
}

// Directions and case byte of vertex j recomputed from g; c receives the
// change of each case count (modulo 2^32), and j's label tile is flagged if
// its direction changed.
template <int NDIM>
__device__ __forceinline__ void refresh_vertex(const EngField& F, int j, bool sum, unsigned (&c)[4]) {
    const unsigned dg = steepest_at<NDIM>(F.g, F.gr, j);
    const unsigned now = case_bits(F.dirs_f[j], dg), was = F.cases[j];
    if (dg != F.dirs_g[j]) F.tile_dirty[tile_of_vertex<NDIM>(F.gr, j)] = 1;
    F.dirs_g[j] = static_cast<uint8_t>(dg);
    F.cases[j] = static_cast<uint8_t>(now);
    if (sum && now != was) {  // the chunk's case counts: types 0, 1 in word 0, types 2, 3 in word 1 (16 bits each)
        const int d0 = static_cast<int>(now & 1u) - static_cast<int>(was & 1u);
        const int d1 = static_cast<int>((now >> 1) & 1u) - static_cast<int>((was >> 1) & 1u);
        const int d2 = static_cast<int>((now >> 2) & 1u) - static_cast<int>((was >> 2) & 1u);
        const int d3 = static_cast<int>((now >> 3) & 1u) - static_cast<int>((was >> 3) & 1u);
        unsigned* w = F.chunk_cnt + 2 * (j >> kEngChunkShift);
        if (d0 | d1) atomicAdd(w, static_cast<unsigned>(d0 + d1 * 65536));
        if (d2 | d3) atomicAdd(w + 1, static_cast<unsigned>(d2 + d3 * 65536));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] += ((now >> t) & 1u) - ((was >> t) & 1u);
}

// ----------------------------------------------------- byte accounting ---
// With profiling on, every step reports the algorithmic bytes of the units
// its blocks visited (per unit, the compulsory reads and writes of the
// operation; halo and cache re-reads are not counted):
//   validate 16 B per vertex (20 with a warm start), directions of f 5,
//   full direction and case pass over g 9, label tile 9 per vertex of a
//   relabelled tile plus 10 per saved face vertex (16 per restored one of an
//   unchanged tile), labels of f 16 per vertex of a visited tile,
//   troublemakers 2 per vertex of a visited tile plus 8 per vertex whose
//   labels are resolved in a direction that differs (16 per direction of a
//   4-vertex group in the start field's count), both plus 4 per gather
//   along an exit chain, 16 per edit attempt and 1 per neighbour flagged
//   after a change; deltas 16; an
//   apply or refresh 1 per flag byte of a chunk it reads (an apply reads only
//   chunks that may hold a case of its type, a refresh only chunks an edit
//   touched) and 12 (apply) or 4 (refresh) per chunk summary, plus 16 per
//   edit attempt and 1 per neighbour flagged after a change (apply) or 9 per
//   recomputed vertex and 32 per cleared flag word (refresh); the compression
//   4 per pointer load or store of its walks and root records.

// Vertices of the direction work items [lo, hi) of F.
template <int NDIM>
__device__ __forceinline__ long long dirs_vertices(const EngField& F, int lo, int hi) {
    const DirsVariant v = variant_of(NDIM, F.variant);
    const Grid& gr = F.gr;
    const int tx = (gr.nx + kTileX - 1) / kTileX, ty = (gr.ny + v.ty - 1) / v.ty;
    const int zc = NDIM == 3 ? v.zc : 1;
    long long n = 0;
    for (int it = lo; it < hi; ++it) {
        const int x0 = (it % tx) * kTileX, y0 = ((it / tx) % ty) * v.ty, z0 = NDIM == 3 ? (it / (tx * ty)) * zc : 0;
        n += static_cast<long long>(min(kTileX, gr.nx - x0)) * min(v.ty, gr.ny - y0) * (NDIM == 3 ? min(zc, gr.nz - z0) : 1);
    }
    return n;
}

// Vertices of label tile t.
template <int NDIM>
__device__ __forceinline__ long long tile_vertices(const Grid& gr, int t) {
    using T = LabelTile<NDIM>;
    const int3 o = tile_origin<NDIM>(gr, t);
    return static_cast<long long>(min(T::X, gr.nx - o.x)) * min(T::Y, gr.ny - o.y) * min(T::Z, gr.nz - o.z);
}

// Vertices of the chunks [lo, hi).
__device__ __forceinline__ long long chunk_vertices(const Grid& gr, int lo, int hi) {
    const long long a = static_cast<long long>(lo) * kEngChunk;
    const long long b = min(static_cast<long long>(hi) * kEngChunk, static_cast<long long>(gr.n));
    return b > a ? b - a : 0;
}

// acct: this thread's share of the algorithmic bytes of the range (see above).
// SUM: keep and use the chunk summaries of the flag arrays where the field
// asks for them (F.sum: the one-field kernel on a field whose blocks scan
// long ranges of chunks; a batch step sizes its blocks' shares for a full
// scan and waits for the slowest, so skipping chunks gains it nothing).
template <int NDIM, bool SUM>
__device__ __forceinline__ void eng_run_range(const EngField& F, const EngState& st, int lo, int hi, char* smem,
                                              unsigned* cnt, unsigned long long& acct) {
    constexpr int NS = NDIM == 3 ? 14 : 6;
    const bool lead = threadIdx.x == 0;  // adds the bytes that are fixed per range
    const bool sum = SUM && F.sum != 0;  // this field keeps chunk summaries
    const Grid& gr = F.gr;
    int* su = reinterpret_cast<int*>(smem);
    int* sd = su + 4096;
    float* sm = reinterpret_cast<float*>(smem);
    const int cidx[4] = {kCntCase + 0, kCntCase + 1, kCntCase + 2, kCntCase + 3};
    switch (st.op) {
        case kOpPreA: {
            unsigned bad = 0;
            const int ng = (gr.n + 3) >> 2;
            for (int item = lo; item < hi; ++item)
                for (int k = 0; k < kEngChunk / 1024; ++k) {
                    const int w = item * (kEngChunk / 4) + threadIdx.x + 256 * k;
                    if (w < ng) validate_group(F.f, F.fhat, F.warm, F.xi, gr.n, F.L, F.g, w, bad);
                }
            if (bad) atomicOr(cnt + kCntErr, bad);
            if (lead) acct += (F.warm ? 20 : 16) * chunk_vertices(gr, lo, hi);
            break;
        }
        case kOpPreA2: {
            unsigned c[4] = {0u, 0u, 0u, 0u};
            eng_dirs<NDIM, 0>(F, F.f, F.dirs_f, lo, hi, sm, c);
            if (lead) acct += 5 * dirs_vertices<NDIM>(F, lo, hi);
            break;
        }
        case kOpPreB:  // the pointers of f's forests, kept for the troublemaker passes
            for (int item = lo; item < hi; ++item) {
                label_tile_body<NDIM>(F.dirs_f, gr, item, F.Mf, F.mf, su, sd);
                __syncthreads();
                if (lead) acct += 9 * tile_vertices<NDIM>(gr, item);
            }
            break;
        case kOpRTile:
            // only tiles with a changed direction are redone: the others'
            // pointers are still those of their last pass
            for (int item = lo; item < hi; ++item) {
                if (!F.tile_dirty[item]) continue;
                label_tile_body<NDIM>(F.dirs_g, gr, item, F.qu, F.qd, su, sd);
                __syncthreads();
                if (threadIdx.x == 0) {
                    F.tile_dirty[item] = 0;
                    acct += 9 * tile_vertices<NDIM>(gr, item);
                }
            }
            break;
        case kOpPreD: {  // f's labels, in place: each pointer becomes the root at the end of its chain
            unsigned bad = 0, hops = 0;
            for (int item = lo; item < hi; ++item) {
                bad |= label_final_tile<NDIM>(F.Mf, F.mf, gr, item, F.Mf, F.mf, hops);
                if (lead) acct += 16 * tile_vertices<NDIM>(gr, item);
            }
            acct += 4ull * hops;
            if (bad) atomicOr(cnt + kCntErr, bad);
            break;
        }
        case kOpApplyC: {
            // the targets of the cases of the current type
            unsigned changed = 0, tries = 0;
            int* list = reinterpret_cast<int*>(smem);
            const int type = st.type;
            int scanned = 0;  // chunks whose case bytes were read
            if (type == kTypeMerged) {
                // every case of every type; all targets claimed, so a vertex
                // proposed by several cases is edited once (or, preemptive,
                // edited by each case that gets there, racing)
                const bool pre = F.preempt != 0;
                const Dirty dirty = dirty_of(F, sum);
                scanned = for_flagged<true>(
                    F.cases, gr.n, lo, hi, 0x0F0F0F0Fu, sum, list, list + kEngChunk,
                    [&](int c) { return F.chunk_unk[c] != 0u || (F.chunk_cnt[2 * c] | F.chunk_cnt[2 * c + 1]) != 0u; },
                    chunk_counted(F),
                    [&](int i) {
                        const unsigned b = F.cases[i];
                        tries += __popc(b & 0xFu);
                        if (b & 9u) target_edit<NDIM>(pre, F.marks, F.g, F.L, dirty, gr, i, changed);
                        if (b & 2u)
                            target_edit<NDIM>(pre, F.marks, F.g, F.L, dirty, gr, i + slot_offset(gr, F.dirs_f[i] & 15u),
                                              changed);
                        if (b & 4u)
                            target_edit<NDIM>(pre, F.marks, F.g, F.L, dirty, gr, i + slot_offset(gr, F.dirs_g[i] >> 4),
                                              changed);
                    },
                    [](int) {});
                if (lead) acct += 12ull * (hi - lo) + static_cast<unsigned long long>(scanned) * kEngChunk;
                acct += 16ull * tries + static_cast<unsigned long long>(NS) * changed;
                unsigned v[1] = {changed};
                const int idx[1] = {kCntChanged};
                block_add<1>(v, cnt, idx);
                break;
            }
            const Dirty dirty = dirty_of(F, sum);
            scanned = for_flagged<true>(
                F.cases, gr.n, lo, hi, 0x01010101u << type, sum, list, list + kEngChunk,
                [&](int c) {
                    return F.chunk_unk[c] != 0u || ((F.chunk_cnt[2 * c + (type >> 1)] >> (16 * (type & 1))) & 0xFFFFu);
                },
                chunk_counted(F),
                [&](int i) {
                    ++tries;
                    if (type == 0 || type == 3) {
                        edit_vertex<NDIM>(F.g, F.L, dirty, gr, i, changed);
                        return;
                    }
                    // FPmin and FNmax targets may be shared
                    const int t = i + slot_offset(gr, type == 1 ? (F.dirs_f[i] & 15u) : (F.dirs_g[i] >> 4));
                    claim_edit<NDIM>(F.marks, F.g, F.L, dirty, gr, t, changed);
                },
                [](int) {});
            if (lead) acct += 12ull * (hi - lo) + static_cast<unsigned long long>(scanned) * kEngChunk;
            acct += 16ull * tries + static_cast<unsigned long long>(NS) * changed;
            unsigned v[1] = {changed};
            const int idx[1] = {kCntChanged};
            block_add<1>(v, cnt, idx);
            break;
        }
        case kOpPreE:
        case kOpFullC:
        case kOpFullR: {
            unsigned c[4] = {0u, 0u, 0u, 0u};
            eng_dirs<NDIM, 1>(F, F.g, F.dirs_g, lo, hi, sm, c);
            block_add<4>(c, cnt, cidx);
            if (lead) acct += 9 * dirs_vertices<NDIM>(F, lo, hi);
            // every label tile is redone next time: this range's share of the flags
            const long long nt = label_tiles_of(gr), items = eng_items(F, st.op);
            for (long long t = lo * nt / items + threadIdx.x; t < hi * nt / items; t += blockDim.x) F.tile_dirty[t] = 1;
            // and every refresh flag is cleared, every case byte rewritten:
            // this range's share of the chunk summaries (counts unknown until
            // the next apply reads the chunk)
            const long long nc = (gr.n + kEngChunk - 1) / kEngChunk;
            for (long long t = lo * nc / items + threadIdx.x; sum && t < hi * nc / items; t += blockDim.x) {
                F.chunk_dirty[t] = 0u;
                F.chunk_unk[t] = 1u;
            }
            break;
        }
        case kOpRefreshC:
        case kOpRefreshR: {
            // directions and cases of the flagged vertices; their flags and
            // marks are cleared
            unsigned c[4] = {0u, 0u, 0u, 0u};
            unsigned nv = 0, nw = 0;
            int* list = reinterpret_cast<int*>(smem);
            const int scanned = for_flagged<false>(
                F.dirty, gr.n, lo, hi, 0xFFFFFFFFu, sum, list, list + kEngChunk,
                [&](int c) { return F.chunk_dirty[c] != 0u; },
                [&](int c, unsigned, unsigned) { F.chunk_dirty[c] = 0u; },
                [&](int j) {
                    refresh_vertex<NDIM>(F, j, sum, c);
                    ++nv;
                },
                [&](int w) {
                    reinterpret_cast<uint4*>(F.dirty)[w] = make_uint4(0u, 0u, 0u, 0u);
                    reinterpret_cast<uint4*>(F.marks)[w] = make_uint4(0u, 0u, 0u, 0u);
                    ++nw;
                });
            block_add<4>(c, cnt, cidx);
            acct += 9ull * nv + 32ull * nw;
            if (lead) acct += 4ull * (hi - lo) + static_cast<unsigned long long>(scanned) * kEngChunk;
            break;
        }
        case kOpRDetect: {
            // Every tile is visited (its labels follow the exit chains, which
            // may run through any relabelled tile).  The
            // troublemakers' targets of the block's tiles go to an LDS list
            // and are edited together once it is half full and at the end
            // (type 0; type 1 only counts): detection reads directions and
            // labels, never g.
            __shared__ unsigned s_targets;
            unsigned wrong = 0, cases = 0, changed = 0;
            const TargetList tl{st.type == 0 ? reinterpret_cast<int*>(smem) : nullptr, &s_targets, F.marks, F.g,
                                F.L, dirty_of(F, sum), F.preempt != 0};
            // the listed targets, edited by all threads; ends with a barrier
            unsigned tries = 0;
            auto edit_targets = [&]() {
                const int nt = min(static_cast<int>(s_targets), TargetList::kCap);
                for (int e = threadIdx.x; e < nt; e += blockDim.x) {
                    target_edit<NDIM>(tl.preempt, F.marks, F.g, F.L, tl.dirty, gr, tl.list[e], changed);
                    ++tries;
                }
                __syncthreads();
            };
            // the troublemaker candidates of a tile: the upper half of the LDS
            __shared__ unsigned s_cand;
            unsigned short* cand_up = reinterpret_cast<unsigned short*>(smem + kEngSmemBytes / 2);
            unsigned short* cand_dn = cand_up + 4096;
            static_assert(kEngSmemBytes / 2 >= 2 * 4096 * sizeof(unsigned short), "candidate lists fit");
            if (threadIdx.x == 0) s_targets = 0, s_cand = 0;
            __syncthreads();
            unsigned bad = 0, hops = 0;
            for (int item = lo; item < hi; ++item) {
                // the start field's count needs every mislabelled vertex;
                // the loop's rounds need only the troublemakers
                if (st.init)
                    detect_r_tile<NDIM>(F.dirs_f, F.dirs_g, F.qu, F.qd, F.Mf, F.mf, gr, item, true,
                                        F.flabels != 0, tl, wrong, cases, changed, bad, hops, acct);
                else
                    detect_r_tile_sparse<NDIM>(F.dirs_f, F.dirs_g, F.qu, F.qd, F.Mf, F.mf, gr, item, tl, cand_up,
                                               cand_dn, &s_cand, cases, changed, bad, hops, acct);
                if (lead) acct += 2 * tile_vertices<NDIM>(gr, item);
                __syncthreads();  // every wave's additions to the list are in s_targets
                // past half the list: edit what it holds and empty it
                if (tl.list && s_targets > TargetList::kCap / 2) {
                    edit_targets();
                    if (threadIdx.x == 0) s_targets = 0;
                    __syncthreads();
                }
            }
            if (tl.list) {
                __syncthreads();
                edit_targets();
            }
            acct += 16ull * tries + static_cast<unsigned long long>(NS) * changed + 4ull * hops;
            if (bad) atomicOr(cnt + kCntErr, bad);
            unsigned v[3] = {wrong, cases, changed};
            const int idx[3] = {kCntWrong, kCntRCases, kCntChanged};
            block_add<3>(v, cnt, idx);
            break;
        }
        case kOpDelta: {
            unsigned edited = 0, inexact = 0;
            const int ng = (gr.n + 3) >> 2;
            for (int item = lo; item < hi; ++item)
                for (int k = 0; k < kEngChunk / 1024; ++k) {
                    const int w = item * (kEngChunk / 4) + threadIdx.x + 256 * k;
                    if (w < ng) delta_group(F.g, F.fhat, gr.n, F.edits, F.g_out, w, edited, inexact);
                }
            if (lead) acct += 16 * chunk_vertices(gr, lo, hi);
            unsigned v[2] = {edited, inexact};
            const int idx[2] = {kCntEdited, kCntInexact};
            block_add<2>(v, cnt, idx);
            break;
        }
        default:
            break;
    }
    __syncthreads();  // the next range reuses the LDS
}

// Profiling record of a step (ts: kEngStampWords zeroed words, or NULL): block
// 0 stores its start in ts[0]; every block raises ts[1 + blockIdx % 64] to its
// end (64 slots keep the atomics from queueing on one address) and adds the
// algorithmic bytes it visited to ts[kEngBytesWord] (one atomic per wave).
// Times come from the constant-rate GPU clock.
__device__ __forceinline__ void stamp_end(unsigned long long* ts, unsigned long long acct) {
    unsigned long long b = acct;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(ts + kEngBytesWord, b);
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(ts + 1 + blockIdx.x % kEngEndSlots, static_cast<unsigned long long>(wall_clock64()));
}

// The schedule (the host loop of a single correction, step by step): the next
// state of one field from the counters of its finished step.  The current case
// counts live in S->cases: a full pass sets them, a refresh adds its changes.
// An apply step is followed by a refresh of the vertices around its edits, or
// by a full pass when so many values changed that streaming the whole field is
// cheaper (the outcome is the same either way).
__device__ __forceinline__ EngState eng_decide(const EngField& F, EngState st, EngStats* S,
                                                const unsigned (&c)[kCntSlots]) {
    auto go = [&](int op) {
        st.op = op;
        st.items = eng_items(F, op);
        return st;
    };
    auto finish = [&](int status) {  // output the deltas, then stop
        S->status = status;
        return go(kOpDelta);
    };
    auto stop = [&](int status) {    // stop without output (invalid input, device error)
        S->status = status;
        return go(kOpDone);
    };
    // the case count of type t, by selects (no dynamic indexing of local
    // arrays, which would go to private memory)
    auto cases_of = [&](int t) {
        return t == 0 ? S->cases[0] : t == 1 ? S->cases[1] : t == 2 ? S->cases[2] : S->cases[3];
    };
    auto set_cases = [&](bool full) {
        for (int t = 0; t < 4; ++t)
            S->cases[t] = (full ? 0 : S->cases[t]) + static_cast<int>(c[kCntCase + t]);
    };
    // C loop: the current type while it has cases, then the next types in
    // turn, back to FPmax while any of the first three has cases; then labels.
    auto c_decide = [&]() {
        if (F.merged) {  // one type: all of them
            st.type = kTypeMerged;
            if (S->cases[0] + S->cases[1] + S->cases[2] + S->cases[3] > 0)
                return S->rounds_total >= F.cap ? finish(MSZ_ENOCONV) : go(kOpApplyC);
            return go(kOpRTile);
        }
        for (int guard = 0; guard < 8; ++guard) {
            if (cases_of(st.type) > 0) return S->rounds_total >= F.cap ? finish(MSZ_ENOCONV) : go(kOpApplyC);
            if (st.type < 3) {
                st.type += 1;
            } else if (S->cases[0] + S->cases[1] + S->cases[2] > 0) {
                st.type = 0;
            } else {
                break;
            }
        }
        return go(kOpRTile);
    };
    // refresh around the changed vertices, or a full pass when they (and
    // their neighbours) would cover more than a quarter of the field
    auto after_apply = [&](int sparse, int full) {
        const long long ring = F.gr.ndim == 3 ? 15 : 7;
        return go(static_cast<long long>(c[kCntChanged]) * ring * 4 > F.gr.n ? full : sparse);
    };
    switch (st.op) {
        case kOpStart:
            return go(kOpPreA);
        case kOpPreA:
            if (c[kCntErr] & kErrNonFinite) return stop(MSZ_ENONFINITE);
            if (c[kCntErr] & kErrBound) return stop(MSZ_EBOUND);
            if (c[kCntErr] & kErrWarmNonFinite) return stop(MSZ_ENONFINITE);
            if (c[kCntErr] & kErrWarmBound) return stop(MSZ_EBOUND);
            return go(kOpPreA2);
        case kOpPreA2:
            return go(kOpPreB);
        case kOpPreB:  // f's labels: resolved once, or followed where the troublemaker passes need them
            st.type = 0;
            return go(F.flabels ? kOpPreD : kOpPreE);
        case kOpPreD:
            if (c[kCntErr] & kErrWalk) return stop(MSZ_EDEVICE);
            return go(kOpPreE);
        case kOpPreE:
            set_cases(true);
            for (int t = 0; t < 4; ++t) S->false_init[t] = c[kCntCase + t];
            S->outer_iters = 1;
            st.type = 0;
            if (F.count_init) {  // labels of the start field, then their count (no edits)
                st.init = 1;
                return go(kOpRTile);
            }
            return c_decide();
        case kOpRefreshC:
        case kOpFullC:
            set_cases(st.op == kOpFullC);
            return c_decide();
        case kOpApplyC:
            if (c[kCntChanged] == 0) return finish(MSZ_ESTALL);
            S->rounds_total += 1;
            if (st.type == kTypeMerged) {  // the types that had cases in this round
                for (int t = 0; t < 4; ++t) S->rounds[t] += S->cases[t] > 0 ? 1 : 0;
            } else if (st.type == 0) S->rounds[0] += 1;
            else if (st.type == 1) S->rounds[1] += 1;
            else if (st.type == 2) S->rounds[2] += 1;
            else S->rounds[3] += 1;
            return after_apply(kOpRefreshC, kOpFullC);
        case kOpRTile:
            // at the cap, and for the start field's count: detect without editing
            st.type = (st.init || S->rounds_total >= F.cap) ? 1 : 0;
            return go(kOpRDetect);
        case kOpRDetect:
            if (c[kCntErr] & kErrWalk) return stop(MSZ_EDEVICE);
            if (st.init) {  // the start field's count; the correction starts now
                S->mislabel_init = c[kCntWrong];
                st.init = 0;
                st.type = 0;
                return c_decide();
            }
            // no troublemaker exactly when no vertex is mislabelled (the
            // detection of the rounds counts only the former)
            if (c[kCntRCases] == 0) return finish(MSZ_OK);
            if (st.type != 0) return finish(MSZ_ENOCONV);
            if (c[kCntChanged] == 0) return finish(MSZ_ESTALL);
            S->rounds_total += 1;
            S->rounds_r += 1;
            st.type = 0;
            return after_apply(kOpRefreshR, kOpFullR);
        case kOpRefreshR:
        case kOpFullR:
            set_cases(st.op == kOpFullR);
            if (S->cases[0] + S->cases[1] + S->cases[2] + S->cases[3] > 0) {
                S->outer_iters += 1;
                return c_decide();
            }
            return go(kOpRTile);
        case kOpDelta:
            S->n_edited = c[kCntEdited];
            S->n_inexact = c[kCntInexact];
            return go(kOpDone);
        default:
            return go(kOpDone);
    }
}

// One step of one chain of a batch (its 2D or its 3D fields, all of
// dimension NDIM), schedule included, in one kernel.  pre[0..nf] are the
// prefix sums of the blocks given to each field in this step and pre[nf + 1]
// the number of fields given blocks; block b runs one contiguous share of the
// items of the field whose blocks contain b (a block never spans two fields:
// a loop over fields around the operations cost the kernel a third of its
// occupancy in registers).  The last block of a field to finish takes the
// field's decision (its next state, from the counters its blocks left), and
// the last field to be decided forms the next step's prefix sums in pre_next
// (cost-weighted: a field gets ceil(units / per) blocks, units = items *
// eng_weight and per = the chain's units over (grid - nf) blocks, rounded up;
// at most the grid in all) and clears the chain's done word once no field has
// items.  tick[f] counts the finished blocks of field f and tick[nf] the
// decided fields; the block that draws the last ticket resets it.
//
// Blocks hand counters, tickets and decided states to each other inside the
// kernel through device-scope atomics only (every XCD sees one value of each),
// and a block draws its ticket after its own memory operations have
// completed: a device-scope fence, which on MI355X writes back the L2 of the
// XCD, is never needed.  Everything else a step writes is read by later
// steps, after the kernel boundary.
__device__ __forceinline__ int ld_dev(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_dev(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// True in every thread of the block that draws ticket n - 1 of *ticket.
__device__ __forceinline__ bool draw_last(int* ticket, int n, int* s_flag) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores and atomics have completed
    __syncthreads();
    if (threadIdx.x == 0)
        *s_flag = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == n - 1;
    __syncthreads();
    return *s_flag != 0;
}

// The decision of field F after its step (all its blocks have finished): the
// 256 threads reduce and clear its counter block, thread 0 runs the schedule.
__device__ __forceinline__ void decide_field(const EngField& F, const EngState& st, EngStats* stats_f,
                                             EngState* nxt_f, int* oplog_f, unsigned* part, unsigned* red) {
    unsigned* cnt = F.cnt;
    const int k = threadIdx.x % kCntSlots, s0 = threadIdx.x / kCntSlots;
    constexpr int PER = kSlots / (256 / kCntSlots);
    unsigned v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = ld_dev(cnt + (s0 + q * (256 / kCntSlots)) * kSlotStride + k);
    unsigned acc = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        acc = k == kCntErr ? (acc | v[q]) : acc + v[q];
        cnt[(s0 + q * (256 / kCntSlots)) * kSlotStride + k] = 0u;  // read next by the step after the next
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < kCntSlots) {
        unsigned a = 0;
        for (int j = threadIdx.x; j < 256; j += kCntSlots) a = threadIdx.x == kCntErr ? (a | part[j]) : a + part[j];
        red[threadIdx.x] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        EngStats S = *stats_f;
        unsigned c[kCntSlots];
        for (int j = 0; j < kCntSlots; ++j) c[j] = red[j];
        const EngState ns = eng_decide(F, st, &S, c);
        *stats_f = S;
        st_dev(&nxt_f->op, ns.op);
        st_dev(&nxt_f->type, ns.type);
        st_dev(&nxt_f->items, ns.items);
        st_dev(&nxt_f->init, ns.init);
        if (oplog_f) *oplog_f = st.op;
    }
}

// The next step's blocks per field (the first wave of the block that decided
// the chain's last field; su: kEngMaxFields words of LDS).  Lane l takes the
// fields l, l + 64, ...; a field no block ran (done) carries its state over.
__device__ __forceinline__ void scan_chain(const EngField* __restrict__ fields, const EngState* cur, EngState* nxt,
                                           const int* pre, int* pre_next, int nf, int* word, int* oplog, int step,
                                           long long* su) {
    const int lane = threadIdx.x;
    long long total = 0;
#pragma unroll 1
    for (int f = lane; f < nf; f += 64) {
        int op, items;
        if (pre[f + 1] == pre[f]) {
            const EngState s = cur[f];
            nxt[f] = s;
            if (oplog) oplog[step * nf + f] = kOpDone;
            op = s.op;
            items = s.items;
        } else {
            op = ld_dev(&nxt[f].op);
            items = ld_dev(&nxt[f].items);
        }
        su[f] = static_cast<long long>(items) * eng_weight(fields[f], op);
        total += su[f];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o, 64);
    const long long slots = static_cast<int>(gridDim.x) > nf ? static_cast<int>(gridDim.x) - nf : 1;
    const long long per = total > 0 ? (total + slots - 1) / slots : 1;
    int carry = 0, act = 0;
#pragma unroll 1
    for (int base = 0; base < nf; base += 64) {
        const int f = base + lane;  // the lane that stored su[f]
        const int nb = f < nf ? static_cast<int>((su[f] + per - 1) / per) : 0;
        int incl = nb;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (f < nf) pre_next[f + 1] = carry + incl;
        carry += __shfl(incl, 63, 64);
        act += __popcll(__ballot(nb > 0));
    }
    if (lane == 0) {
        pre_next[0] = 0;
        pre_next[nf + 1] = act;
        // the done word lives in pinned host memory, which the host polls
        if (total == 0) __hip_atomic_store(word, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int NDIM>
__global__ void __launch_bounds__(256) k_eng_step(const EngField* __restrict__ fields, const EngState* cur,
                                                  EngState* nxt, EngStats* stats, const int* pre, int* pre_next,
                                                  int nf, int* tick, int* word, int* oplog, int step,
                                                  unsigned long long* ts) {
    __shared__ __align__(16) char smem[kEngSmemBytes];
    __shared__ int s_flag;
    static_assert(3 * DirsGeom<3, 32, 16>::P * sizeof(float) <= sizeof(smem), "stencil planes fit the LDS");
    static_assert(kEngMaxFields * sizeof(long long) <= sizeof(smem), "the chain's units fit the LDS");
    if (ts && blockIdx.x == 0 && threadIdx.x == 0) ts[0] = static_cast<unsigned long long>(wall_clock64());
    unsigned long long acct = 0;
    // the tables were written by the previous steps, so plain loads see them
    const int used = pre[nf];
    const int b = xcd_logical_block(blockIdx.x, gridDim.x);
    if (used == 0) {
        // the chain is done (the rest of this graph launch): carry the states over
        if (b == 0) {
            for (int f = threadIdx.x; f < nf; f += blockDim.x) {
                nxt[f] = cur[f];
                if (oplog) oplog[step * nf + f] = kOpDone;
            }
            if (threadIdx.x == 0) pre_next[nf] = 0, pre_next[nf + 1] = 0;
        }
    } else if (b < used) {
        int a = 0, z = nf - 1;  // the field whose blocks contain b: largest f with pre[f] <= b
        while (a < z) {
            const int mid = (a + z + 1) >> 1;
            if (pre[mid] <= b) a = mid;
            else z = mid - 1;
        }
        const EngState st = cur[a];
        const int nbf = pre[a + 1] - pre[a];
        const long long j = b - pre[a];
        const int i0 = static_cast<int>(j * st.items / nbf), i1 = static_cast<int>((j + 1) * st.items / nbf);
        if (i0 < i1) eng_run_range<NDIM, false>(fields[a], st, i0, i1, smem, fields[a].cnt, acct);
        if (draw_last(tick + a, nbf, &s_flag)) {
            unsigned* part = reinterpret_cast<unsigned*>(smem);
            decide_field(fields[a], st, stats + a, nxt + a, oplog ? oplog + step * nf + a : nullptr, part,
                         part + 256);
            if (threadIdx.x == 0) st_dev(tick + a, 0);
            if (draw_last(tick + nf, pre[nf + 1], &s_flag)) {
                if (threadIdx.x < 64)
                    scan_chain(fields, cur, nxt, pre, pre_next, nf, word, oplog, step,
                               reinterpret_cast<long long*>(smem));
                if (threadIdx.x == 0) st_dev(tick + nf, 0);
            }
        }
    }
    if (ts) stamp_end(ts, acct);
}

// One field, one kernel per step: every block takes the schedule decision
// itself (the same one: the same inputs, the same arithmetic) from the state
// and statistics of step k - 1 and the counters that step left, then runs its
// range of the chosen operation.  Buffers by step: states and stats by k % 2
// (a step reads k - 1's and block 0 writes k's); counter sets by k % 3 (a step
// reads set k - 1, adds into set k and clears set k + 1, which step k - 1
// read and step k + 1 fills).  stats[2] receives the statistics once the
// field is done; then the final statistics go to the done word block hflag
// (pinned host memory, or device memory for the no-allocation entry point;
// skipped when NULL) and its first word is cleared.  A
// graph holds kEngTimeSlots (a multiple of 6) steps, so the parities continue
// across launches.
template <int NDIM>
__global__ void __launch_bounds__(256) k_eng_step1(const EngField* __restrict__ fields, EngState* states,
                                                   const EngState* __restrict__ states_in, EngStats* stats,
                                                   unsigned* cnt3, int* ctl, int* hflag, int* oplog, int k,
                                                   unsigned long long* ts) {
    __shared__ __align__(16) char smem[kEngSmemBytes];
    __shared__ unsigned part[256];
    __shared__ unsigned red[kCntSlots];
    __shared__ EngState s_next;
    __shared__ EngStats s_stats;
    static_assert(kEngTimeSlots % 6 == 0, "parities of 2 and 3 continue across graph launches");
    static_assert(sizeof(EngStats) % 4 == 0 && sizeof(EngStats) / 4 <= 256, "statistics copied word by word");
    if (ts && blockIdx.x == 0 && threadIdx.x == 0) ts[0] = static_cast<unsigned long long>(wall_clock64());
    const int p = k & 1;
    unsigned* c_prev = cnt3 + ((k + 2) % 3) * kCntBlockWords;
    unsigned* c_cur = cnt3 + (k % 3) * kCntBlockWords;
    unsigned* c_next = cnt3 + ((k + 1) % 3) * kCntBlockWords;
    // all loads first: the state of step k - 1 (a scalar load: states_in is
    // the same array, read-only here, as this step writes only states[p]),
    // its counters and statistics
    const EngState prev = states_in[p ^ 1];
    const int kc = threadIdx.x % kCntSlots, s0 = threadIdx.x / kCntSlots;
    constexpr int PER = kSlots / (256 / kCntSlots);
    unsigned v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = c_prev[(s0 + q * (256 / kCntSlots)) * kSlotStride + kc];
    if (prev.items == 0 && prev.op != kOpStart) {
        // the field is done (the rest of this graph launch): carry the state over
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            states[p] = prev;
            ctl[0] = 0;
            if (oplog) oplog[k] = kOpDone;
        }
        return;
    }
    constexpr int SW = sizeof(EngStats) / 4;
    if (threadIdx.x < SW)  // the statistics of step k - 1, word by word into LDS
        reinterpret_cast<unsigned*>(&s_stats)[threadIdx.x] = reinterpret_cast<const unsigned*>(stats + (p ^ 1))[threadIdx.x];
    unsigned acc = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) acc = kc == kCntErr ? (acc | v[q]) : acc + v[q];
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < kCntSlots) {
        unsigned a = 0;
        for (int j = threadIdx.x; j < 256; j += kCntSlots) a = threadIdx.x == kCntErr ? (a | part[j]) : a + part[j];
        red[threadIdx.x] = a;
    }
    __syncthreads();
    const EngField& F = fields[0];
    if (threadIdx.x == 0) {
        EngState ns = prev;
        if (prev.items > 0 || prev.op == kOpStart) {
            unsigned c[kCntSlots];
            for (int j = 0; j < kCntSlots; ++j) c[j] = red[j];
            ns = eng_decide(F, prev, &s_stats, c);
        }
        s_next = ns;
        if (blockIdx.x == 0) {
            states[p] = ns;
            stats[p] = s_stats;
            if (ns.items == 0) stats[2] = s_stats;
            ctl[0] = ns.items > 0 ? 1 : 0;
            if (ns.items == 0 && hflag) {
                // the final statistics, then the done word, into pinned host
                // memory (the host waits for the word to drop to 0)
                constexpr int SW = sizeof(EngStats) / 4;
                unsigned* hs = reinterpret_cast<unsigned*>(hflag) + kHostStatsWord;
                for (int w = 0; w < SW; ++w)
                    __hip_atomic_store(hs + w, reinterpret_cast<const unsigned*>(&s_stats)[w], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(hflag, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            if (oplog) oplog[k] = ns.items > 0 ? ns.op : kOpDone;
        }
    }
    // clear the counter set of step k + 1 (read by step k - 1, filled by step k + 1)
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < kCntBlockWords; w += gridDim.x * blockDim.x) c_next[w] = 0u;
    __syncthreads();
    const EngState st = s_next;
    unsigned long long acct = 0;
    if (st.items > 0) {
        const int nb = gridDim.x, b = xcd_logical_block(blockIdx.x, nb);
        const int per = (st.items + nb - 1) / nb;
        const int lo = b * per, hi = min(st.items, lo + per);
        if (lo < hi) eng_run_range<NDIM, true>(F, st, lo, hi, smem, c_cur, acct);
    }
    if (ts) stamp_end(ts, acct);
}

// Start of a one-field run: the field table entry (passed by value), the
// states of "step -1" (done) and step 0 (start), the three counter sets, the
// statistics, the active word, the done word (when it lives in device memory,
// else NULL: the host raises its own) and the field's marks, case bytes and
// dirty flags -- everything the host would otherwise upload or clear one
// call at a time.
__global__ void __launch_bounds__(256) k_eng_setup1(const EngField F, EngField* fields, EngState* states,
                                                    EngStats* stats, unsigned* cnt3, int* ctl, int* done_word) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nthr = gridDim.x * blockDim.x;
    if (tid == 0) {
        fields[0] = F;
        states[0] = EngState{kOpDone, 0, 0, 0};
        states[1] = EngState{kOpStart, 0, 1, 0};
        ctl[0] = 1;
        if (done_word) done_word[0] = 1;
    }
    for (int w = tid; w < 3 * kCntBlockWords; w += nthr) cnt3[w] = 0u;
    constexpr int SW = 3 * static_cast<int>(sizeof(EngStats) / 4);
    for (int w = tid; w < SW; w += nthr) reinterpret_cast<unsigned*>(stats)[w] = 0u;
    const int nw = (F.gr.n + 15) >> 4;
    for (int w = tid; w < nw; w += nthr) {
        reinterpret_cast<uint4*>(F.marks)[w] = make_uint4(0u, 0u, 0u, 0u);
        reinterpret_cast<uint4*>(F.cases)[w] = make_uint4(0u, 0u, 0u, 0u);
        reinterpret_cast<uint4*>(F.dirty)[w] = make_uint4(0u, 0u, 0u, 0u);
    }
    const int nc = (F.gr.n + kEngChunk - 1) / kEngChunk;
    for (int c = tid; c < nc; c += nthr) {
        F.chunk_dirty[c] = F.chunk_cnt[2 * c] = F.chunk_cnt[2 * c + 1] = 0u;
        F.chunk_unk[c] = 1u;
    }
}

// Clears every field's marks, case bytes, dirty flags, their chunk summaries
// and counter block.
__global__ void __launch_bounds__(256) k_eng_init(const EngField* __restrict__ fields, int nf) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nthr = gridDim.x * blockDim.x;
    for (int f = 0; f < nf; ++f) {
        const EngField& F = fields[f];
        uint4* m = reinterpret_cast<uint4*>(F.marks);
        uint4* cs = reinterpret_cast<uint4*>(F.cases);
        uint4* dt = reinterpret_cast<uint4*>(F.dirty);
        const int nw = (F.gr.n + 15) >> 4;
        for (int w = tid; w < nw; w += nthr) {
            m[w] = make_uint4(0u, 0u, 0u, 0u);
            cs[w] = make_uint4(0u, 0u, 0u, 0u);
            dt[w] = make_uint4(0u, 0u, 0u, 0u);
        }
        const int nc = (F.gr.n + kEngChunk - 1) / kEngChunk;
        for (int c = tid; c < nc; c += nthr) {
            F.chunk_dirty[c] = F.chunk_cnt[2 * c] = F.chunk_cnt[2 * c + 1] = 0u;
            F.chunk_unk[c] = 1u;
        }
        for (int w = tid; w < kCntBlockWords; w += nthr) F.cnt[w] = 0u;
    }
}

const void* eng_step_kernel(int ndim) {
    return ndim == 3 ? reinterpret_cast<const void*>(&k_eng_step<3>) : reinterpret_cast<const void*>(&k_eng_step<2>);
}
const void* eng_step1_kernel(int ndim) {
    return ndim == 3 ? reinterpret_cast<const void*>(&k_eng_step1<3>) : reinterpret_cast<const void*>(&k_eng_step1<2>);
}
const void* eng_init_kernel() { return reinterpret_cast<const void*>(&k_eng_init); }
const void* eng_setup1_kernel() { return reinterpret_cast<const void*>(&k_eng_setup1); }

}  // namespace msz
