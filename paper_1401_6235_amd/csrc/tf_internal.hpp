// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tf.h"
#include "tf_kernels.hpp"
#include "tf_launch.hpp"

namespace tf {

// Where and how one library call launches its kernels.
struct Launch {
    hipStream_t stream;
    bool aligned;  // every array 16-byte aligned: 128-bit vector path
    int64_t cap;   // cap on the grid in blocks (0 = none)
};

// Process-wide launch settings (tf_config).
struct Config {
    int64_t ew_blocks_per_cu = 0;
    int64_t red_tiles_per_block = 0;  // 0: tuned per element size and leaf kind
    int64_t red_waves = 0;            // waves per first-pass block; 0: tuned
};
Config &config();
int num_cus();

template <typename T>
void run_elementwise(const Launch &L, int op, int64_t n, const void *x0, const void *x1,
                     const void *y0, const void *y1, void *z0, void *z1);
template <typename T>
void run_plain(const Launch &L, int op, int64_t n, const void *x, const void *y, void *z);
template <typename T>
void run_axpy(const Launch &L, int64_t n, const void *a, const void *x0, const void *x1,
              const void *y0, const void *y1, void *z0, void *z1);
template <typename T>
void run_plain_axpy(const Launch &L, int64_t n, const void *a, const void *x, const void *y, void *z);
template <typename T>
void run_horner(const Launch &L, int64_t n, int degree, const void *c, const void *x0, const void *x1,
                void *z0, void *z1);
template <typename T>
void run_plain_horner(const Launch &L, int64_t n, int degree, const void *c, const void *x, void *z);

int chain_code(int op, int mode);
template <typename T>
void run_chain(const Launch &L, int code, int64_t n, int64_t reps, const void *x0, const void *x1,
               const void *y0, const void *y1, void *z0, void *z1);
template <typename T>
void run_plain_chain(const Launch &L, int op, int64_t n, int64_t reps, const void *x, const void *y, void *z);
template <typename T>
void run_trsv(const Launch &L, int64_t nsys, int m, const void *U0, const void *U1, const void *f0,
              const void *f1, void *x0, void *x1);
template <typename T>
void run_plain_trsv(const Launch &L, int64_t nsys, int m, const void *U, const void *f, void *x);
template <typename T>
void run_quadratic(const Launch &L, int64_t n, const void *const *in, void *const *out);
template <typename T>
void run_plain_quadratic(const Launch &L, int64_t n, const void *a, const void *b, const void *c, void *r,
                         void *s);
template <typename T>
void run_fma(const Launch &L, int64_t n, const void *const *in, void *z0, void *z1);
template <typename T>
void run_plain_fma(const Launch &L, int64_t n, const void *x, const void *y, const void *w, void *z);

// Leaf kinds of the reduction tree.
enum Leaf {
    LEAF_SUM_D = 0,   // dotted values; Two-Sum at level 1
    LEAF_SUM_T = 1,   // twofold values (x0, x1)
    LEAF_DOT_DD = 2,  // Two-Product of dotted x, y
    LEAF_DOT_TT = 3,  // MTF1 of twofold x, y
    LEAF_DOT_TD = 4,  // MTF1.1, twofold x, dotted y
    LEAF_DOT_DT = 5,  // MTF1.1, dotted x, twofold y
    LEAF_PSUM = 6,    // plain sum
    LEAF_PDOT = 7,    // plain dot
};

// Geometry of one reduction: tiles of 256 leaves, `per_block` tiles (a
// power of two) per block, `blocks` launched, `padded` = next power of two
// of the tile count divided by per_block (partials beyond `blocks` are
// zero).
struct RedShape {
    int64_t tiles;
    int64_t per_block;
    int64_t blocks;
    int64_t padded;
};
RedShape reduce_shape(int64_t n, int64_t per_block);
// Tiles per first-pass block for this element size and leaf kind: the
// configured value, or the tuned default when none is configured.
int64_t tiles_per_block(int elem_size, int leaf);
// Largest tiles-per-block value a first-pass block handles (64 per wave).
constexpr int64_t kMaxTilesPerBlock = 256;
// Number of (z0, z1) partials a reduction of n leaves at `per_block` tiles
// per block writes to its workspace (0 when it needs none).
int64_t reduce_work_pairs(int64_t n, int64_t per_block);

template <typename T>
void run_reduce(const Launch &L, int leaf, int64_t n, int64_t per_block, const void *x0, const void *x1,
                const void *y0, const void *y1, void *out, void *work);

}  // namespace tf
