// msz_internal.h -- declarations shared by the kernels and the host driver of libmsz.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msz {

constexpr unsigned kSelf = 15u;        // direction slot meaning "the vertex itself"
constexpr int kTileX = 64;             // x extent of a direction tile (16 threads x 4 vertices)
constexpr float kValueLimit = 1.2676506002282294e30f;  // 2^100: inputs above it are rejected

// Round counters.  The device block holds kSlots copies of kCntSlots counters,
// kSlotStride uint32 apart (one 128-byte line each); a launch's blocks add into
// slot blockIdx % kSlots and the host sums the slots (error bits are OR-ed).
constexpr int kSlots = 64;
constexpr int kSlotStride = 32;
constexpr int kCntBlockWords = kSlots * kSlotStride;
constexpr int kGridCap = 2048;  // grid-stride kernels: 8 blocks per compute unit
enum : int {
    kCntCase = 0,      // 0..3: false critical points per C type in the last detection
    kCntChanged = 5,   // values changed by the last apply
    kCntWrong = 6,     // mislabelled vertices (R detection) / wrong_any (compare)
    kCntRCases = 7,    // R-loop troublemaker hits
    kCntErr = 8,       // validation error bits
    kCntEdited = 9,
    kCntInexact = 10,
    kCntWrongMax = 11,
    kCntWrongMin = 12,
    kCntSlots = 16
};
enum : unsigned { kErrNonFinite = 1u, kErrBound = 2u, kErrWarmNonFinite = 4u, kErrWarmBound = 8u, kErrWalk = 16u };

struct Grid {
    int ndim, nx, ny, nz, nxy, n;
    int off[16];  // linear id offset of each neighbour slot; off[15] = 0 (self)
};

int tile_variant_count(int ndim);

void launch_validate_init(const float* f, const float* fhat, const float* warm, float xi, int n,
                          float* L, float* g, unsigned* cnt, hipStream_t s);
void launch_check_finite(const float* h, int n, unsigned* cnt, hipStream_t s);
void launch_dirs(const float* h, const Grid& gr, int variant, uint8_t* dirs_out, hipStream_t s);
void launch_dirs_detect(const float* g, const Grid& gr, int variant, uint8_t* dirs_g,
                        const uint8_t* dirs_f, int type, uint8_t* marks, unsigned* cnt, hipStream_t s);
void launch_detect_only(const uint8_t* dirs_f, const uint8_t* dirs_g, const Grid& gr, int type,
                        uint8_t* marks, unsigned* cnt, hipStream_t s);
void launch_apply(float* g, const float* L, uint8_t* marks, int n, unsigned* cnt, hipStream_t s);
void launch_label_tile(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, hipStream_t s);
void launch_label_compress(const Grid& gr, int* q_up, int* q_dn, unsigned* cnt, hipStream_t s);
void launch_label_forests(const uint8_t* dirs, const Grid& gr, int* q_up, int* q_dn, unsigned* cnt,
                          hipStream_t s);
void launch_label_final(const int* q_up, const int* q_dn, int n, int* M, int* m, hipStream_t s);
void launch_detect_r(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* q_up, const int* q_dn,
                     const int* Mf, const int* mf, const Grid& gr, uint8_t* marks, unsigned* cnt,
                     hipStream_t s);
void launch_compare(const uint8_t* dirs_f, const uint8_t* dirs_g, const int* qfu, const int* qfd,
                    const int* qgu, const int* qgd, int n, unsigned* cnt, hipStream_t s);
void launch_delta(const float* g, const float* fhat, int n, float* delta, float* g_out, unsigned* cnt,
                  hipStream_t s);

}  // namespace msz
