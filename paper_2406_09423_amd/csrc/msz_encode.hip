// msz_encode.hip -- lossless encoding of the edits (Sec. 6.3): the edited
// vertices' indices, sorted, as a gap sequence, and their edit values, each
// stream entropy-coded with a canonical Huffman code, on the GPU.
//
// Stream format (all little-endian; declared with the entry points in msz.h):
//   header (kEncHeader bytes): magic "MSZE", version, n, m, chunk count,
//       edits per chunk, then the code lengths of the 32 gap symbols and of
//       the 512 value symbols (one byte each), zero padding;
//   chunk table: per chunk {uint32 word offset into the bit stream, int32
//       index of the chunk's first edit};
//   bit stream: uint32 words; chunk c starts at its own word.
// Within a chunk the edits follow in index order.  An edit is
//   [gap, for all but the chunk's first edit]  Huffman code of the bucket
//       b = floor(log2(d)) of d = index - previous index (d >= 1), then the b
//       low bits of d (d - 2^b);
//   [value]  Huffman code of the 9 high bits of the float32 edit (sign and
//       exponent), then its 23 mantissa bits.
// Every field is emitted most significant bit first; emitted bit j of a chunk
// is bit (j % 32) of the chunk's word (j / 32).  Huffman codes are canonical
// (symbols ordered by code length, then by symbol) and at most kEncMaxLen bits
// long: the lengths come from the standard two-smallest-merge construction
// (ties broken by node age), and while a length exceeds the limit every count
// is halved (rounding up) and the code rebuilt.
// An edit is a vertex whose edit value is not +0 (the loop only lowers values,
// so every edited vertex has a negative edit).
#include <algorithm>
#include <cstring>
#include <queue>
#include <utility>
#include <vector>

#include "msz_internal.h"

namespace msz {

constexpr int kEncGapSyms = 32, kEncValSyms = 512, kEncMaxLen = 20;
constexpr int kEncChunk = 256;         // edits per chunk (one decoding thread each)
constexpr int kEncBlock = 4096;        // dense entries per compaction block (256 threads x 16)
constexpr int kEncHeader = 576;        // header bytes (24 fixed + 544 code lengths, padded)
constexpr unsigned kEncMagic = 0x455A534Du;  // "MSZE"
constexpr unsigned kEncVersion = 1u;

struct EncCode {  // canonical code of one symbol: the code in its low `len` bits
    unsigned code;
    int len;
};

// ------------------------------------------------------------- kernels ---

__device__ __forceinline__ int gap_bucket(unsigned d) { return 31 - __clz(d); }

// Non-zero edit counts of each block of kEncBlock dense entries.
__global__ void __launch_bounds__(256) k_enc_count(const unsigned* __restrict__ bits, long long n,
                                                   unsigned* __restrict__ counts) {
    __shared__ unsigned part[256];
    const long long base = static_cast<long long>(blockIdx.x) * kEncBlock + 16LL * threadIdx.x;
    unsigned c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) c += (base + k < n && bits[base + k] != 0u) ? 1u : 0u;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = part[0];
}

// In-place exclusive prefix sum of v[0..len) with the total in v[len]
// (one block of 1024 threads walking 1024-element pieces).
__global__ void __launch_bounds__(1024) k_enc_scan(unsigned* v, int len) {
    __shared__ unsigned s[1024];
    __shared__ unsigned carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int p = 0; p < len; p += 1024) {
        const int i = p + threadIdx.x;
        const unsigned x = i < len ? v[i] : 0u;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
            const unsigned y = threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < len) v[i] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) v[len] = carry;
}

// Block-local exclusive scan of 256 thread values (returns the thread's offset).
__device__ __forceinline__ unsigned block_exclusive(unsigned x, unsigned* s) {
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned y = threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    const unsigned r = s[threadIdx.x] - x;
    __syncthreads();
    return r;
}

// The edits of each dense block, in index order, at the block's offset.
__global__ void __launch_bounds__(256) k_enc_compact(const unsigned* __restrict__ bits, long long n,
                                                     const unsigned* __restrict__ offsets, int* __restrict__ idx,
                                                     unsigned* __restrict__ val) {
    __shared__ unsigned s[256];
    const long long base = static_cast<long long>(blockIdx.x) * kEncBlock + 16LL * threadIdx.x;
    unsigned b[16];
    unsigned c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        b[k] = base + k < n ? bits[base + k] : 0u;
        c += b[k] != 0u;
    }
    unsigned o = offsets[blockIdx.x] + block_exclusive(c, s);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (b[k] != 0u) {
            idx[o] = static_cast<int>(base + k);
            val[o] = b[k];
            ++o;
        }
}

// Symbol counts: gap buckets (all but each chunk's first edit) and value symbols.
__global__ void __launch_bounds__(256) k_enc_hist(const int* __restrict__ idx, const unsigned* __restrict__ val,
                                                  int m, unsigned* __restrict__ ghist, unsigned* __restrict__ vhist) {
    __shared__ unsigned g[kEncGapSyms], h[kEncValSyms];
    for (int i = threadIdx.x; i < kEncValSyms; i += blockDim.x) h[i] = 0u;
    if (threadIdx.x < kEncGapSyms) g[threadIdx.x] = 0u;
    __syncthreads();
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        if (k % kEncChunk != 0) atomicAdd(&g[gap_bucket(static_cast<unsigned>(idx[k] - idx[k - 1]))], 1u);
        atomicAdd(&h[val[k] >> 23], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kEncValSyms; i += blockDim.x)
        if (h[i]) atomicAdd(vhist + i, h[i]);
    if (threadIdx.x < kEncGapSyms && g[threadIdx.x]) atomicAdd(ghist + threadIdx.x, g[threadIdx.x]);
}

struct EncTables {
    EncCode gap[kEncGapSyms];
    EncCode val[kEncValSyms];
};

__device__ __forceinline__ int edit_bits(const EncTables& T, const int* idx, const unsigned* val, int k) {
    int nb = T.val[val[k] >> 23].len + 23;
    if (k % kEncChunk != 0) {
        const int b = gap_bucket(static_cast<unsigned>(idx[k] - idx[k - 1]));
        nb += T.gap[b].len + b;
    }
    return nb;
}

// One block per chunk, one thread per edit: bit offsets of the chunk's
// edits and the chunk's length in words (into chunk_words[c]).
static_assert(kEncChunk == 256, "a chunk is one block of 256 threads");
__global__ void __launch_bounds__(256) k_enc_offsets(const EncTables* __restrict__ T, const int* __restrict__ idx,
                                                     const unsigned* __restrict__ val, int m,
                                                     unsigned* __restrict__ bitoff, unsigned* __restrict__ chunk_words) {
    __shared__ unsigned s[256];
    const int k = blockIdx.x * kEncChunk + threadIdx.x;
    const unsigned nb = k < m ? static_cast<unsigned>(edit_bits(*T, idx, val, k)) : 0u;
    const unsigned o = block_exclusive(nb, s);
    if (k < m) bitoff[k] = o;
    if (threadIdx.x == 255) chunk_words[blockIdx.x] = (o + nb + 31) >> 5;
}

// Appends `w` bits of v (most significant first) at bit position pos of a
// 128-bit buffer whose bit j is emitted j-th.
__device__ __forceinline__ void put_bits(unsigned long long (&buf)[2], int& pos, unsigned v, int w) {
    if (w == 0) return;
    const unsigned long long r = static_cast<unsigned long long>(__builtin_bitreverse32(v) >> (32 - w));
    if (pos < 64) {
        buf[0] |= r << pos;
        if (pos + w > 64) buf[1] |= r >> (64 - pos);
    } else {
        buf[1] |= r << (pos - 64);
    }
    pos += w;
}

// Every edit ORs its bits into the (zeroed) stream; neighbouring edits share
// boundary words, hence the atomics.
__global__ void __launch_bounds__(256) k_enc_write(const EncTables* __restrict__ T, const int* __restrict__ idx,
                                                   const unsigned* __restrict__ val, int m,
                                                   const unsigned* __restrict__ bitoff,
                                                   const unsigned* __restrict__ chunk_word0,
                                                   unsigned* __restrict__ stream) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        unsigned long long buf[2] = {0ull, 0ull};
        int pos = 0;
        if (k % kEncChunk != 0) {
            const unsigned d = static_cast<unsigned>(idx[k] - idx[k - 1]);
            const int b = gap_bucket(d);
            put_bits(buf, pos, T->gap[b].code, T->gap[b].len);
            put_bits(buf, pos, d - (1u << b), b);
        }
        const unsigned v = val[k];
        put_bits(buf, pos, T->val[v >> 23].code, T->val[v >> 23].len);
        put_bits(buf, pos, v & 0x7FFFFFu, 23);
        const unsigned start = bitoff[k];
        const unsigned sh = start & 31u;
        unsigned* w = stream + chunk_word0[k / kEncChunk] + (start >> 5);
        // the buffer shifted by sh: at most 31 + 93 bits, four words
        const unsigned long long lo = buf[0] << sh;
        const unsigned long long mid = sh ? (buf[0] >> (64 - sh)) | (buf[1] << sh) : buf[1];
        const unsigned out[4] = {static_cast<unsigned>(lo), static_cast<unsigned>(lo >> 32),
                                 static_cast<unsigned>(mid), static_cast<unsigned>(mid >> 32)};
        const int nw = static_cast<int>((sh + pos + 31) >> 5);
        for (int q = 0; q < nw; ++q)
            if (out[q]) atomicOr(w + q, out[q]);
    }
}

// Chunk table entries: word offset and first index of every chunk.
__global__ void __launch_bounds__(256) k_enc_table(const int* __restrict__ idx, const unsigned* __restrict__ word0,
                                                   int nchunks, unsigned* __restrict__ table) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunks) return;
    table[2 * c] = word0[c];
    table[2 * c + 1] = static_cast<unsigned>(idx[c * kEncChunk]);
}

// Canonical decoding tables: for each length L, the first code, the number
// of codes, and the offset of its symbols in the symbol list.
struct DecTable {
    int first[kEncMaxLen + 1], count[kEncMaxLen + 1], offset[kEncMaxLen + 1];
    int sym[kEncValSyms];
};
struct DecTables {
    DecTable gap, val;
};

// Reads one chunk's bits in stream order (bit j of the chunk is bit j % 32 of
// its word j / 32).  Words arrive eight at a time through a register queue
// (eight independent loads per memory round trip instead of one dependent
// load per word); 33 to 64 bits wait in buf, so a field of up to 30 bits or a
// code of up to 20 is taken with shifts and one bit reversal (fields are
// emitted most significant bit first).  Bits past the chunk's last word read
// as zeros and mark the read as over.
struct BitReader {
    const unsigned* w;
    unsigned next, end;      // next word to load, end of the chunk's words
    unsigned long long buf;  // the next `have` bits, the next one in bit 0
    int have;
    unsigned q0, q1, q2, q3, q4, q5, q6, q7;  // loaded words, q0 first
    int qn;
    long long used, limit;   // bits taken, bits in the chunk
    bool over;
    __device__ __forceinline__ void init(const unsigned* words, unsigned w0, unsigned wend) {
        w = words;
        next = w0;
        end = wend;
        buf = 0ull;
        have = 0;
        q0 = q1 = q2 = q3 = q4 = q5 = q6 = q7 = 0u;
        qn = 0;
        used = 0;
        limit = 32ll * (wend - w0);
        over = false;
    }
    __device__ __forceinline__ void fetch() {
        const unsigned left = end > next ? end - next : 0u;
        const int k = left < 8u ? static_cast<int>(left) : 8;
        q0 = k > 0 ? w[next] : 0u;
        q1 = k > 1 ? w[next + 1] : 0u;
        q2 = k > 2 ? w[next + 2] : 0u;
        q3 = k > 3 ? w[next + 3] : 0u;
        q4 = k > 4 ? w[next + 4] : 0u;
        q5 = k > 5 ? w[next + 5] : 0u;
        q6 = k > 6 ? w[next + 6] : 0u;
        q7 = k > 7 ? w[next + 7] : 0u;
        qn = k;
        next += static_cast<unsigned>(k);
    }
    __device__ __forceinline__ unsigned pop() {
        if (qn == 0) fetch();
        if (qn == 0) return 0u;  // past the chunk
        const unsigned v = q0;
        q0 = q1, q1 = q2, q2 = q3, q3 = q4, q4 = q5, q5 = q6, q6 = q7, q7 = 0u;
        --qn;
        return v;
    }
    __device__ __forceinline__ void fill() {
        while (have <= 32) {
            buf |= static_cast<unsigned long long>(pop()) << have;
            have += 32;
        }
    }
    __device__ __forceinline__ void skip(int n) {
        buf >>= n;
        have -= n;
        used += n;
        if (used > limit) over = true;
    }
    // the next n <= 30 bits as a number (first bit most significant)
    __device__ __forceinline__ unsigned bits(int n) {
        if (n == 0) return 0u;
        fill();
        const unsigned v = __brev(static_cast<unsigned>(buf)) >> (32 - n);
        skip(n);
        return v;
    }
};

// -1 on a malformed stream.
__device__ __forceinline__ int decode_symbol(const DecTable& t, BitReader& r) {
    r.fill();
    const unsigned peek = __brev(static_cast<unsigned>(r.buf));  // the next 32 bits, first one on top
    for (int len = 1; len <= kEncMaxLen; ++len) {
        const int rel = static_cast<int>(peek >> (32 - len)) - t.first[len];
        if (rel >= 0 && rel < t.count[len]) {
            r.skip(len);
            return t.sym[t.offset[len] + rel];
        }
    }
    return -1;
}

// One thread per chunk: decodes its edits and writes them into the dense
// (zeroed) output.  Malformed input (a bad code, an index outside [0, n), a
// read past the chunk) sets *bad.  The code tables are staged in LDS.
__global__ void __launch_bounds__(64) k_dec_chunks(const DecTables* __restrict__ Tg, const unsigned* __restrict__ table,
                                                   const unsigned* __restrict__ stream, unsigned stream_words,
                                                   int nchunks, int m, long long n, unsigned* __restrict__ out,
                                                   unsigned* __restrict__ bad) {
    __shared__ DecTables T_s;
    static_assert(sizeof(DecTables) % 4 == 0, "tables copied word by word");
    for (int i = threadIdx.x; i < static_cast<int>(sizeof(DecTables) / 4); i += blockDim.x)
        reinterpret_cast<unsigned*>(&T_s)[i] = reinterpret_cast<const unsigned*>(Tg)[i];
    __syncthreads();
    const DecTables* T = &T_s;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nchunks) return;
    const unsigned w0 = table[2 * c];
    const unsigned wend = c + 1 < nchunks ? table[2 * (c + 1)] : stream_words;
    if (w0 > wend || wend > stream_words) {
        atomicOr(bad, 1u);
        return;
    }
    BitReader r;
    r.init(stream, w0, wend);
    const int k_end = min(m, (c + 1) * kEncChunk);
    long long i = static_cast<int>(table[2 * c + 1]);
    for (int k = c * kEncChunk; k < k_end; ++k) {
        if (k != c * kEncChunk) {
            const int b = decode_symbol(T->gap, r);
            if (b < 0 || b > 30) {
                atomicOr(bad, 1u);
                return;
            }
            i += static_cast<long long>((1u << b) + r.bits(b));
        }
        const int e = decode_symbol(T->val, r);
        const unsigned mant = r.bits(23);
        if (e < 0 || r.over || i < 0 || i >= n) {
            atomicOr(bad, 1u);
            return;
        }
        out[i] = (static_cast<unsigned>(e) << 23) | mant;
    }
}

__global__ void __launch_bounds__(256) k_enc_fill(unsigned* p, long long nw, unsigned v) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < nw; i += static_cast<long long>(gridDim.x) * 256)
        p[i] = v;
}

// ------------------------------------------------------------ host side ---

// Code lengths of a Huffman code for the counts (0 for absent symbols): the
// two lightest nodes merge first, ties going to the older node (leaves are
// older than internal nodes and ordered by symbol); while the longest code
// exceeds kEncMaxLen every count is halved, rounding up, and the code rebuilt.
std::vector<int> huffman_lengths(std::vector<unsigned long long> f) {
    const int ns = static_cast<int>(f.size());
    std::vector<int> len(ns, 0);
    int present = 0, last = -1;
    for (int s = 0; s < ns; ++s)
        if (f[s]) ++present, last = s;
    if (present == 0) return len;
    if (present == 1) {
        len[last] = 1;
        return len;
    }
    for (;;) {
        typedef std::pair<unsigned long long, int> Node;  // (weight, id): leaves 0..ns-1, then merges
        std::priority_queue<Node, std::vector<Node>, std::greater<Node>> q;
        std::vector<int> parent(2 * ns, -1);
        for (int s = 0; s < ns; ++s)
            if (f[s]) q.push(Node(f[s], s));
        int next = ns;
        while (q.size() > 1) {
            const Node a = q.top();
            q.pop();
            const Node b = q.top();
            q.pop();
            parent[a.second] = next;
            parent[b.second] = next;
            q.push(Node(a.first + b.first, next));
            ++next;
        }
        int longest = 0;
        for (int s = 0; s < ns; ++s) {
            if (!f[s]) continue;
            int d = 0;
            for (int x = s; parent[x] >= 0; x = parent[x]) ++d;
            len[s] = d;
            longest = std::max(longest, d);
        }
        if (longest <= kEncMaxLen) return len;
        for (unsigned long long& x : f)
            if (x) x = (x + 1) >> 1;
    }
}

// Canonical codes from code lengths (symbols ordered by length, then symbol).
void canonical_codes(const std::vector<int>& len, EncCode* out) {
    const int ns = static_cast<int>(len.size());
    std::vector<int> order;
    for (int s = 0; s < ns; ++s)
        if (len[s]) order.push_back(s);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return len[a] != len[b] ? len[a] < len[b] : a < b; });
    unsigned code = 0;
    int prev = order.empty() ? 0 : len[order[0]];
    for (int s = 0; s < ns; ++s) out[s] = EncCode{0u, 0};
    for (size_t k = 0; k < order.size(); ++k) {
        const int s = order[k];
        code <<= (len[s] - prev);
        prev = len[s];
        out[s] = EncCode{code, len[s]};
        ++code;
    }
}

void decode_table(const uint8_t* len, int ns, DecTable& t) {
    std::memset(&t, 0, sizeof(t));
    std::vector<int> order;
    for (int s = 0; s < ns; ++s)
        if (len[s]) order.push_back(s);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return len[a] != len[b] ? len[a] < len[b] : a < b; });
    for (size_t k = 0; k < order.size(); ++k) t.sym[k] = order[k];
    unsigned code = 0;
    int pos = 0;
    for (int L = 1; L <= kEncMaxLen; ++L) {
        int cnt = 0;
        for (int s = 0; s < ns; ++s) cnt += len[s] == L;
        t.first[L] = static_cast<int>(code);
        t.count[L] = cnt;
        t.offset[L] = pos;
        pos += cnt;
        code = (code + cnt) << 1;
    }
}

size_t enc_bound(long long n, long long m) {
    const long long chunks = (m + kEncChunk - 1) / kEncChunk;
    const long long edit_bits_max = kEncMaxLen + 30 + kEncMaxLen + 23;
    return static_cast<size_t>(kEncHeader + 8 * chunks + 4 * (chunks + (m * edit_bits_max + 31) / 32));
}

}  // namespace msz

using namespace msz;

extern "C" {

size_t msz_edits_bound(int64_t n) {
    if (n < 0 || n >= (int64_t(1) << 31)) return 0;
    return enc_bound(n, n);
}

int msz_encode_edits(const float* edits, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                     msz_edit_stats* st, void* stream) {
    if (!edits || !out || !out_bytes || n < 0 || n >= (int64_t(1) << 31)) return MSZ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(edits) & 15u) || (reinterpret_cast<uintptr_t>(out) & 15u)) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned* bits = reinterpret_cast<const unsigned*>(edits);
    const int nblocks = static_cast<int>((n + kEncBlock - 1) / kEncBlock);
    // scratch: block offsets (+ total), indices, values, bit offsets, chunk words (+ total), histograms, tables
    const size_t m_max = static_cast<size_t>(n);
    const size_t nchunks_max = (m_max + kEncChunk - 1) / kEncChunk;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += (b + 255) & ~size_t(255);
        return r;
    };
    const size_t o_off = take(4 * (nblocks + 1)), o_idx = take(4 * m_max), o_val = take(4 * m_max),
                 o_bit = take(4 * m_max), o_cw = take(4 * (nchunks_max + 1)), o_hist = take(4 * (kEncGapSyms + kEncValSyms)),
                 o_tab = take(sizeof(EncTables)), o_bad = take(4);
    (void)o_bad;
    char* scratch = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&scratch), std::max<size_t>(o, 256), s) != hipSuccess) return MSZ_ENOMEM;
    auto fail = [&](int rc) {
        (void)hipFreeAsync(scratch, s);
        (void)hipStreamSynchronize(s);
        return rc;
    };
    unsigned* off = reinterpret_cast<unsigned*>(scratch + o_off);
    int* idx = reinterpret_cast<int*>(scratch + o_idx);
    unsigned* val = reinterpret_cast<unsigned*>(scratch + o_val);
    unsigned* bitoff = reinterpret_cast<unsigned*>(scratch + o_bit);
    unsigned* cw = reinterpret_cast<unsigned*>(scratch + o_cw);
    unsigned* hist = reinterpret_cast<unsigned*>(scratch + o_hist);
    EncTables* tab = reinterpret_cast<EncTables*>(scratch + o_tab);
    unsigned m = 0;
    if (nblocks > 0) {
        hipLaunchKernelGGL(k_enc_count, dim3(nblocks), dim3(256), 0, s, bits, static_cast<long long>(n), off);
        hipLaunchKernelGGL(k_enc_scan, dim3(1), dim3(1024), 0, s, off, nblocks);
        if (hipMemcpyAsync(&m, off + nblocks, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MSZ_EDEVICE);
    }
    // word offsets are 32-bit: the stream of m edits (at most 93 bits each) must fit
    if (static_cast<unsigned long long>(m) * 93ull / 32ull + static_cast<unsigned long long>(m) / kEncChunk + 2 >
        0xFFFFFFFFull)
        return fail(MSZ_EINVAL);
    const int nchunks = static_cast<int>((m + kEncChunk - 1) / kEncChunk);
    std::vector<unsigned> h(kEncGapSyms + kEncValSyms, 0u);
    if (m > 0) {
        hipLaunchKernelGGL(k_enc_compact, dim3(nblocks), dim3(256), 0, s, bits, static_cast<long long>(n), off, idx,
                           val);
        hipLaunchKernelGGL(k_enc_fill, dim3(1), dim3(256), 0, s, hist, static_cast<long long>(kEncGapSyms + kEncValSyms),
                           0u);
        const int hb = std::min(1024, static_cast<int>((m + 255) / 256));
        hipLaunchKernelGGL(k_enc_hist, dim3(hb), dim3(256), 0, s, idx, val, static_cast<int>(m), hist,
                           hist + kEncGapSyms);
        if (hipMemcpyAsync(h.data(), hist, 4 * h.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MSZ_EDEVICE);
    }
    std::vector<unsigned long long> fg(h.begin(), h.begin() + kEncGapSyms), fv(h.begin() + kEncGapSyms, h.end());
    const std::vector<int> lg = huffman_lengths(fg), lv = huffman_lengths(fv);
    EncTables ht;
    canonical_codes(lg, ht.gap);
    canonical_codes(lv, ht.val);
    unsigned words = 0;
    if (m > 0) {
        if (hipMemcpyAsync(tab, &ht, sizeof(ht), hipMemcpyHostToDevice, s) != hipSuccess) return fail(MSZ_EDEVICE);
        hipLaunchKernelGGL(k_enc_offsets, dim3(nchunks), dim3(256), 0, s, tab, idx, val, static_cast<int>(m), bitoff, cw);
        hipLaunchKernelGGL(k_enc_scan, dim3(1), dim3(1024), 0, s, cw, nchunks);
        if (hipMemcpyAsync(&words, cw + nchunks, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MSZ_EDEVICE);
    }
    const size_t bytes = static_cast<size_t>(kEncHeader) + 8ull * nchunks + 4ull * words;
    *out_bytes = bytes;
    if (bytes > capacity) return fail(MSZ_EINVAL);
    std::vector<uint8_t> head(kEncHeader, 0);
    const unsigned fixed[6] = {kEncMagic, kEncVersion, static_cast<unsigned>(n), m, static_cast<unsigned>(nchunks),
                               static_cast<unsigned>(kEncChunk)};
    std::memcpy(head.data(), fixed, sizeof(fixed));
    for (int i = 0; i < kEncGapSyms; ++i) head[24 + i] = static_cast<uint8_t>(lg[i]);
    for (int i = 0; i < kEncValSyms; ++i) head[24 + kEncGapSyms + i] = static_cast<uint8_t>(lv[i]);
    char* ob = static_cast<char*>(out);
    if (hipMemcpyAsync(ob, head.data(), kEncHeader, hipMemcpyHostToDevice, s) != hipSuccess) return fail(MSZ_EDEVICE);
    if (m > 0) {
        unsigned* table = reinterpret_cast<unsigned*>(ob + kEncHeader);
        unsigned* sw = reinterpret_cast<unsigned*>(ob + kEncHeader + 8ull * nchunks);
        hipLaunchKernelGGL(k_enc_table, dim3((nchunks + 255) / 256), dim3(256), 0, s, idx, cw, nchunks, table);
        hipLaunchKernelGGL(k_enc_fill, dim3(std::max(1u, std::min(2048u, (words + 255) / 256))), dim3(256), 0, s, sw,
                           static_cast<long long>(words), 0u);
        hipLaunchKernelGGL(k_enc_write, dim3(std::min(4096, static_cast<int>((m + 255) / 256))), dim3(256), 0, s, tab,
                           idx, val, static_cast<int>(m), bitoff, cw, sw);
    }
    if (hipGetLastError() != hipSuccess) return fail(MSZ_EDEVICE);
    if (st) {
        st->n = n;
        st->n_edits = m;
        st->bytes = static_cast<int64_t>(bytes);
        st->index_bits = 0;
        st->value_bits = 0;
        // split of the stream bits by field, from the symbol counts and code lengths
        for (int b = 0; b < kEncGapSyms; ++b) st->index_bits += static_cast<int64_t>(h[b]) * (lg[b] + b);
        for (int e = 0; e < kEncValSyms; ++e) st->value_bits += static_cast<int64_t>(h[kEncGapSyms + e]) * (lv[e] + 23);
    }
    (void)hipFreeAsync(scratch, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSZ_EDEVICE;
    return MSZ_OK;
}

int msz_decode_edits(const void* in, size_t in_bytes, float* edits_out, int64_t n, void* stream) {
    if (!in || !edits_out || n < 0 || n >= (int64_t(1) << 31) || in_bytes < static_cast<size_t>(kEncHeader))
        return MSZ_EINVAL;
    if ((reinterpret_cast<uintptr_t>(in) & 15u) || (reinterpret_cast<uintptr_t>(edits_out) & 15u)) return MSZ_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint8_t> head(kEncHeader);
    if (hipMemcpyAsync(head.data(), in, kEncHeader, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MSZ_EDEVICE;
    unsigned fixed[6];
    std::memcpy(fixed, head.data(), sizeof(fixed));
    const unsigned m = fixed[3], nchunks = fixed[4];
    if (fixed[0] != kEncMagic || fixed[1] != kEncVersion || fixed[2] != static_cast<unsigned>(n) ||
        fixed[5] != static_cast<unsigned>(kEncChunk) || nchunks != (m + kEncChunk - 1) / kEncChunk || m > fixed[2])
        return MSZ_EINVAL;
    if (in_bytes < static_cast<size_t>(kEncHeader) + 8ull * nchunks) return MSZ_EINVAL;
    const size_t stream_words = (in_bytes - kEncHeader - 8ull * nchunks) / 4;
    DecTables dt;
    for (int i = 0; i < kEncGapSyms + kEncValSyms; ++i)
        if (head[24 + i] > kEncMaxLen) return MSZ_EINVAL;
    decode_table(head.data() + 24, kEncGapSyms, dt.gap);
    decode_table(head.data() + 24 + kEncGapSyms, kEncValSyms, dt.val);
    char* scratch = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&scratch), 512 + sizeof(DecTables), s) != hipSuccess) return MSZ_ENOMEM;
    unsigned* bad = reinterpret_cast<unsigned*>(scratch);
    DecTables* tp = reinterpret_cast<DecTables*>(scratch + 256);
    unsigned* outw = reinterpret_cast<unsigned*>(edits_out);
    hipLaunchKernelGGL(k_enc_fill, dim3(1), dim3(256), 0, s, bad, 1LL, 0u);
    hipLaunchKernelGGL(k_enc_fill, dim3(std::max(1, std::min(4096, static_cast<int>((n + 255) / 256)))), dim3(256), 0, s,
                       outw, static_cast<long long>(n), 0u);
    unsigned hbad = 0;
    int rc = MSZ_OK;
    if (hipMemcpyAsync(tp, &dt, sizeof(dt), hipMemcpyHostToDevice, s) != hipSuccess) rc = MSZ_EDEVICE;
    if (rc == MSZ_OK && nchunks > 0) {
        const char* ib = static_cast<const char*>(in);
        hipLaunchKernelGGL(k_dec_chunks, dim3((nchunks + 63) / 64), dim3(64), 0, s, tp,
                           reinterpret_cast<const unsigned*>(ib + kEncHeader),
                           reinterpret_cast<const unsigned*>(ib + kEncHeader + 8ull * nchunks),
                           static_cast<unsigned>(stream_words), static_cast<int>(nchunks), static_cast<int>(m),
                           static_cast<long long>(n), outw, bad);
        if (hipGetLastError() != hipSuccess) rc = MSZ_EDEVICE;
    }
    if (rc == MSZ_OK && (hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess)) rc = MSZ_EDEVICE;
    (void)hipFreeAsync(scratch, s);
    if (hipStreamSynchronize(s) != hipSuccess) rc = MSZ_EDEVICE;
    if (rc == MSZ_OK && hbad) rc = MSZ_EINVAL;
    return rc;
}

}  // extern "C"
