// Internal declarations of the quantization sweep (not part of the C ABI).
#pragma once

#include "common.h"

namespace mgs {

constexpr int LGTAB = 256;            // h * log2(h) table entries kept in LDS
constexpr int MGS_MAX_ENTRIES = 40;   // histogram windows per plan
constexpr int REPL_WORDS = 1024;      // words a replicated low-b histogram may take (G / 8 if more)
constexpr int REPL_MAX_LOG = 5;       // at most 32 copies per bin
constexpr int MGS_XCDS = 8;           // XCDs that workgroups are dispatched over, round-robin

// One histogram window of one bit-width inside a batch of LDS words.
struct HistEntry {
    // Every field is a 4-byte word, so that the kernel reads an entry with
    // scalar loads (sub-word fields at unaligned offsets become vector loads
    // whose latency each wavefront waits out once per entry).
    int32_t bi;       // index into the bit-width list
    int32_t b;        // the bit-width (every scene of a launch has the same list)
    int32_t packed;   // two 16-bit bins per 32-bit word
    int32_t first;    // first window of this b: it also accumulates the loss
    int32_t split;    // the b's bins span more than one window
    int32_t rtn;      // entropy from the atomics' old counts (no scan of the bins)
    int32_t rlog;     // log2 of the copies per bin (lane-interleaved replicas)
    int32_t lo;       // first word of the window within the b's words
    int32_t nwords;   // words in the window
    int32_t lds_off;  // word offset of the window inside the batch
};

// Everything the kernels need to know about one scene's sweep.
struct SceneDesc {
    const float* attr;
    const float* imp;
    const int32_t* kept;
    double* err;
    double* bits;
    float* gmin;
    float* gmax;
    uint32_t* hist;
    int32_t* order;                 // [gpc]: the run's groups in tile order (workspace)
    int64_t ld;
    int64_t hist_bins;              // sum over the list of 2^b
    int32_t C, T, G, nb;
    int32_t gmaxn;                  // group slots per (t, c) in the tables
    int32_t gpc;                    // real groups per channel, sum_t ceil(k_t / G)
    int32_t bmax;
    int32_t pad;
    int64_t k[MGS_MAX_RATIOS];
    int64_t koff[MGS_MAX_RATIOS];
    int32_t gcum[MGS_MAX_RATIOS + 1];  // prefix of ceil(k_t / G) over t
    int32_t pad2;
    int64_t hoff[MGS_MAX_BITS];        // debug-histogram offset of each b
    uint8_t bl[MGS_MAX_BITS];
};

// Kernel arguments shared by all tiles of one launch.
struct SweepParams {
    mgs_status_block* status;
    const SceneDesc* scenes;  // device array (workspace)
    const double* lgtab;      // T(h) = h log2 h for h in [0, lgtab_max], then the increments
                              // F[c] = R(T(c+1)) - R(T(c)), R: rounding to the grid 2^-K
    int64_t ntiles;
    int64_t tcum[MGS_MAX_JOBS + 1];  // prefix of the tiles of each scene
    int32_t nscenes;
    int32_t lgtab_max;
    int32_t cpb;              // channels per tile
    int32_t nbatches, nentries, max_batch_words;
    int32_t kgrid;            // K of the increment grid
    int32_t persist;          // persistent grid: tiles from the per-XCD counters of status->queue
    // split tail (all channels per tile, persistent): each XCD's range of
    // tper tile indices covers tgpx groups of the scenes' tile orders in
    // sequence, the last tranks of them as tparts runs of tcpb channels; tcum
    // then holds the prefix of the scenes' groups
    int32_t tsplit, tcpb, tparts;
    int64_t tgpx, tranks, tper;
    int32_t batch_begin[MGS_MAX_ENTRIES + 1];
    int32_t batch_words[MGS_MAX_ENTRIES];
    int32_t batch_scan_end[MGS_MAX_ENTRIES];  // a batch's scanned entries come first: [begin, scan_end)
    HistEntry entries[MGS_MAX_ENTRIES];
};

// Launch shape and LDS capacity of the sweep kernel.
struct Shape {
    int nt;        // threads per workgroup
    int ept;       // elements per thread (nt * ept >= G, else the chunked kernel)
    int lds_cap;   // LDS bytes the histogram plan may use (0 = device maximum)
    int cpb = 0;   // channels per tile (0 = all channels)
    int persist = 0;  // 1: a persistent grid sized to the resident slots, tiles from per-XCD queues
};

int fill_scene(const mgs_sweep_desc* d, const float* attr, const float* imp, const int32_t* kept,
               double* err, double* bits, float* gmin, float* gmax, uint32_t* hist, SceneDesc* sc);
bool build_plan(const uint8_t* bl, int nb, int cap_words, int G, SweepParams* p);
int plan_for(const SceneDesc& sc, const Shape& sh, SweepParams* p, size_t* lds_bytes);
Shape default_shape(int G, int nb, int bmax);
bool shape_valid(const Shape& sh, int G);
// Copies `count` scene descriptors into device memory and prepares the
// tables (NaN padding, status reset, debug histogram clearing) and each
// scene's tile order (host_scenes[i].order must point at gpc ints).
int launch_init(const SceneDesc* host_scenes, int count, SceneDesc* d_scenes,
                mgs_status_block* status, double* lgtab, int lgtab_max, hipStream_t s);
// Grid exponent K of the entropy increments: every partial sum of up to G
// increments stays an exact FP64 multiple of 2^-K.
int increment_grid_bits(int G);
// G: the largest group size of the launch (selects the chunked kernel when
// it exceeds the shape's nt * ept).
int launch_sweep(const SweepParams& p, const Shape& sh, size_t lds,
                 int64_t grid, hipStream_t s, int G);
int max_resident_blocks(const Shape& sh, size_t lds, int G);
int device_cus();
int variant_count();
Shape variant_shape(int i);
bool variant_chunked(int i);

// Autotune registry: the shape chosen for (G, nb, bmax), if any.
bool tuned_shape(int G, int nb, int bmax, Shape* out);
void set_tuned_shape(int G, int nb, int bmax, const Shape& sh);

}  // namespace mgs
