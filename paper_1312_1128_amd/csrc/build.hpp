// Tree storage owned by a glm_tree handle, and the build entry point.
#pragma once

#include "common.hpp"

namespace glm {

constexpr int kLevReps = 16;

// The particle sort first orders the Morton keys on their top kTopDigits
// 8-bit digits only (which fix the boxes down to level kTopLevel = 16: two
// key bits per level), then orders each
// run of keys equal in those digits by the rest (runs of up to kTieRun keys):
// the full-key order, unless a box at level kTopLevel holds more than L
// particles.  The topology count flags that case
// (BuildSync::deep), and the build then sorts on all 64 bits; a tree that was
// deep at its last build starts with the full sort.
constexpr int kTopDigits = 4;
constexpr int kTieRun = 64;
constexpr int kTopLevel = 4 * kTopDigits;

// radix_sort_u64 on the digits first .. first + passes - 1 only (sort.hip).
int radix_sort_u64_digits(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int first, int passes,
                          uint32_t* hist, hipStream_t s);
static_assert(kMaxLevel + 1 <= 64, "a level-count copy holds 64 levels");

// Small device struct written by the build kernels; copied to the host once.
struct BuildSync {
    double x0, y0, side, scale; // root square and 32-bit quantisation scale
    int32_t ncells;
    int32_t bad;                // input validation flag
    int32_t nleaves;
    int32_t max_level;
    int32_t nlisted;
    int32_t internal;           // consistency flags of the build (0 = ok)
    int32_t deep;               // a box at level kTopLevel holds more than L particles
    int32_t levcnt[kMaxLevel + 2];  // boxes per level
    int32_t levfill[kMaxLevel + 2]; // fill counters of the per-level box index
    // boxes per level counted in kLevReps copies (block b adds into copy
    // b % kLevReps, each in its own 256-byte line), so that the topology
    // blocks' atomics do not all queue on one line; summed into levcnt
    alignas(256) int32_t levrep[kLevReps][64];
};

// Host copy of the per-level layout of the box index.
struct LevelTable {
    int32_t off[kMaxLevel + 2];
    int32_t cnt[kMaxLevel + 2];
};

// Build-side per-box arrays (preorder).
struct BoxArrays {
    int32_t *beg, *end, *level, *next, *leaf;
    uint32_t *ix, *iy;
    int32_t *lbeg, *lend;
};

// Bump layout of one device buffer (256-byte aligned pieces).
struct Arena {
    size_t size = 0;
    size_t take(size_t bytes)
    {
        const size_t o = size;
        size += (bytes + 255) & ~size_t(255);
        return o;
    }
};

// Every device array of a tree lives in the caller's workspace: the
// per-particle part first (its size follows from n), then the per-box part
// (its size from the box count, known after the topology pass).
struct TreeStorage {
    char* ws = nullptr;      // caller's workspace (device), borrowed
    size_t ws_bytes = 0;
    size_t need = 0;         // bytes the last build needed (also after a refusal for space)
    bool built = false;
    int32_t n = 0, ncells = 0;
    glm_params params{};
    double x0 = 0, y0 = 0, side = 0;
    BuildSync* sync = nullptr; // device
    BoxArrays b{};
    int32_t* perm = nullptr;   // Morton position -> original index
    uint64_t* key = nullptr;   // sorted Morton keys
    bool deep = false;         // the last build had a box below level kTopLevel
    double *ccx = nullptr, *ccy = nullptr;
    double* ms = nullptr;      // FP64 masses in Morton order
    TreeDev dev{};
};

// Largest number of boxes a tree of n particles and leaf size L can have:
// leaves are disjoint and non-empty (at most n); an internal box holds more
// than L particles, so a level has at most min(4^l, n / (L + 1)) of them
// (levels 0..31); and a tree with I internal boxes has at most 4 I + 1.
int64_t max_boxes(int64_t n, int L);
// Bytes of the per-particle part and of the per-box part of a tree.
size_t tree_particle_bytes(int64_t n);
size_t tree_box_bytes(int64_t ncells, int order);

// Build into ts.ws (ws_bytes >= tree_particle_bytes(n)); GLM_ENOMEM when the
// boxes do not fit after it (ts.need then holds the bytes required).
glm_status build_tree_device(TreeStorage& ts, const double* x, const double* y, const double* m, const double* s,
                             int64_t n, const glm_params& prm, hipStream_t st);

// Smoothing lengths of the tree's particles (knn.hip): distance to the k-th
// nearest other particle, written in original order.
glm_status knn_device(const TreeStorage& ts, int k, double* s_out, hipStream_t st);

// Smoothing lengths from raw positions (knn3.hip): 2D (z NULL) or 3D, and per
// species when species is not NULL; the caller's workspace holds
// knn_workspace_bytes(n, species != NULL) bytes.  Synchronises the stream
// once (twice with species) to validate the inputs and read the species
// segments.
size_t knn_workspace_bytes(int64_t n, bool species);
glm_status knn_positions_device(const double* x, const double* y, const double* z, const int32_t* species,
                                int64_t n, int k, double* s_out, void* ws, hipStream_t st);

} // namespace glm
