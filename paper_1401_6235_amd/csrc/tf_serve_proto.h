/*
 * Serving protocol between the host server and the persistent kernel.
 *
 * Host-coherent memory (pinned, fine-grained) holds a ring of job
 * descriptors written by the host and one completion record per slot
 * written by the device.  Device memory holds the slot table the workers
 * claim from.  Plain C so the host server, the kernel and a CPU stand-in
 * for the device (used by the host-logic tests) share one definition.
 *
 * Publication: the host fills ring[seq % TFS_RING] for a free slot, then
 * stores pub_count = seq + 1 with release semantics.  The kernel's
 * dispatcher wave reads pub_count with acquire (system scope), copies each
 * new descriptor into the device slot table and opens the slot by a
 * release store of its control word.  A job whose inputs are generated on
 * the device opens in the generation phase: its units first write the
 * inputs, and the block that finishes the last of them reopens the slot in
 * the compute phase.
 *
 * Completion: the worker that finishes a job's last claim writes the
 * job's done record, its `gen` field last with a system-scope release;
 * the host reads `gen` with acquire and then the rest of the record.
 */
#ifndef TF_SERVE_PROTO_H
#define TF_SERVE_PROTO_H

#include <stdint.h>

#include "tf.h" /* TFS_MAX_SLOTS, TFS_OP_*, TFS_KIND_* */

#define TFS_RING 256           /* descriptor ring entries (power of two) */
#define TFS_CLAIM 4096         /* elements per claimed unit of work */
#define TFS_MAX_CLAIMS 16383   /* claims per job (14-bit field) */
#define TFS_MAX_N ((int64_t)TFS_CLAIM * TFS_MAX_CLAIMS)
#define TFS_MAX_BATCH 16       /* units claimed by one fetch-add, at most */

/* Control word of a device slot: generation (low 32 bits of the
 * publication number, never 0), phase (1 bit: TFS_PHASE_GEN or
 * TFS_PHASE_COMPUTE), number of units in the phase (14 bits), next
 * unclaimed unit (17 bits).  gen == 0: slot empty.  Workers claim with a
 * fetch-add of 1 .. TFS_MAX_BATCH units; a worker adds only after it has
 * seen next < units, so the count runs past the number of units by at most
 * TFS_MAX_BATCH times the number of workers (at most 1024:
 * 16383 + 16 x 1024 < 2^17) and never reaches the units field. */
#define TFS_PHASE_COMPUTE 0
#define TFS_PHASE_GEN 1
#define TFS_CTL(gen, phase, ntiles, next)                                                          \
    (((uint64_t)(uint32_t)(gen) << 32) | ((uint64_t)(phase) << 31) | ((uint64_t)(ntiles) << 17) | \
     (uint64_t)(next))
#define TFS_CTL_GEN(c) ((c) >> 32)
#define TFS_CTL_PHASE(c) (((c) >> 31) & 1u)
#define TFS_CTL_NTILES(c) (((c) >> 17) & 0x3fffu)
#define TFS_CTL_NEXT(c) ((c)&0x1ffffu)
#ifdef __cplusplus
static_assert(TFS_MAX_CLAIMS <= 0x3fff, "unit count fits its 14-bit field");
static_assert(TFS_MAX_CLAIMS + TFS_MAX_BATCH * 1024 <= 0x1ffff,
              "next unit plus the overshoot of 1024 workers fits its 17-bit field");
#endif

typedef struct {
    uint64_t gen;      /* publication number, 1, 2, ... */
    int32_t slot;      /* device slot */
    int32_t op;        /* TFS_OP_* */
    int32_t dtype;     /* TF_F32 / TF_F64 */
    int32_t kind;      /* TFS_KIND_* */
    int64_t n;
    uint64_t seed;
    int32_t degree;    /* Horner degree */
    int32_t nclaims;   /* claims of TFS_CLAIM elements */
    int32_t tiles_per_claim; /* reductions: 256-leaf tiles per claim (power of two) */
    int32_t padded;    /* reductions: claims padded to a power of two */
    int32_t ngen;      /* units of TFS_CLAIM elements that generate the inputs (0: provided) */
    int32_t pad0;
    double a0, a1;     /* axpy scalar, already rounded to dtype */
    double thr;        /* flag threshold on |z1| / |z0| */
    double c[33];      /* Horner coefficients, already rounded to dtype */
    uint64_t x0, x1, y0, y1;  /* device addresses of the inputs (0 = absent) */
    uint64_t z0, z1;   /* outputs of vector jobs */
    uint64_t part;     /* per-claim partials */
} tfs_desc;

typedef struct {
    uint64_t gen;          /* publication this record belongs to (written last) */
    int32_t status;
    int32_t flag;
    double z0, z1;         /* scalar jobs (sum, dot), widened to binary64 */
    double max0, max1;     /* vector jobs: max |z0_i|, max |z1_i| */
    uint64_t n_flagged;    /* vector jobs: elements with |z1_i| > thr |z0_i| */
    uint64_t nonfinite;    /* elements (or results) that are not finite */
    uint64_t hash0, hash1; /* vector jobs: sum of the bit patterns, mod 2^64 */
    uint64_t t_open;  /* device wall clock: slot opened by the dispatcher */
    uint64_t t_start; /* first unit claimed */
    uint64_t t_ready; /* inputs generated, compute phase opened (0: provided inputs) */
    uint64_t t_end;   /* record written */
} tfs_done;

/* Host-coherent shared region. */
typedef struct {
    uint64_t pub_count;    /* host: number of descriptors published */
    uint64_t stop;         /* host: 1 = drain and exit */
    uint64_t consumed;     /* device: descriptors copied into slots */
    uint64_t kernel_state; /* device: 1 running, 2 exited normally, 3 idle timeout */
    uint64_t heartbeat;    /* device: dispatcher loop count */
    uint64_t claims_done;  /* device: claims processed (statistics) */
    uint64_t pad[2];
    tfs_desc ring[TFS_RING];
    tfs_done done[TFS_MAX_SLOTS];
} tfs_shared;

/* Per-claim summary of a vector job (device memory). */
typedef struct {
    double max0, max1;
    uint64_t n_flagged, nonfinite, hash0, hash1;
} tfs_vsum;

/* Counter-based input generator: the k-th output of a SplitMix64 stream
 * seeded with s (Steele, Lea and Flood, OOPSLA 2014; the finaliser
 * constants of Vigna's splitmix64), mix(s + (k + 1) * golden gamma).
 * Element i of array a (0: x0, 1: x1, 2: y0, 3: y1) uses k = 4 i + a. */
#define TFS_GAMMA 0x9e3779b97f4a7c15ull
#define TFS_MIX1 0xbf58476d1ce4e5b9ull
#define TFS_MIX2 0x94d049bb133111ebull

#endif /* TF_SERVE_PROTO_H */
