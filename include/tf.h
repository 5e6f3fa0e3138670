/*
 * tf.h - twofold fast arithmetic on AMD Instinct MI355X (gfx950).
 *
 * A twofold is an unevaluated sum z0 + z1 of two floating-point numbers of
 * one working type (E. Latkin, "Twofold fast arithmetic", 2014): z0 is
 * bitwise the standard IEEE result of the operation on the main parts, and
 * z1 approximates its deviation dz0 = z - z0 from the exact result z.  The
 * library evaluates the paper's algorithms elementwise over large arrays
 * and in a few streaming kernels built from them.
 *
 * Data layout: structure of arrays.  A twofold array of n elements is two
 * separate arrays of n values, its main parts (z0) and its error parts (z1).
 * A NULL error-part pointer on an input marks a "dotted" operand (a plain
 * number), which selects the paper's cheaper *.1 / *.1.1 variants.  Outputs
 * always have both parts.
 *
 * Conventions for every call below:
 *   dtype      TF_F64 (binary64, double) or TF_F32 (binary32, float); all
 *              arrays of one call hold that type.
 *   n          number of elements, n >= 0; n == 0 launches nothing
 *              (reductions then write (+0, +0)).
 *   pointers   device pointers (HBM), owned by the caller, unless marked
 *              HOST.  Elementwise calls never allocate.  An output may alias
 *              an input exactly (in place); partial overlap is undefined.
 *              Any natural alignment works; 16-byte alignment of every
 *              array selects the 128-bit vector path.
 *   stream     HIP stream the kernels are enqueued on (0 = null stream).
 *              Calls return once the work is enqueued; results are
 *              visible in stream order.  The library never synchronises.
 *   return     TF_OK, or a negative TF_E* code for misuse (NULL required
 *              pointer, n < 0, unknown dtype, degree out of range, workspace
 *              too small) or a failed launch.  NaN, infinities, division by
 *              zero and square roots of negatives are data, not errors: they
 *              propagate through the basic operations exactly as the paper
 *              prescribes (no special-case handling).
 *
 * Every kernel is built without fast-math, with floating-point contraction
 * off, IEEE division and square root, and denormals kept, so each step is
 * one correctly rounded IEEE operation (round to nearest, ties to even).
 */
#ifndef TF_H
#define TF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Working types. */
#define TF_F32 1
#define TF_F64 2

/* Status codes. */
#define TF_OK 0
#define TF_EINVAL (-1)  /* invalid argument */
#define TF_EDEVICE (-2) /* a HIP call or kernel launch failed */
#define TF_ENOMEM (-3)  /* workspace too small / allocation failed */
#define TF_EBUSY (-4)   /* resource temporarily exhausted (serving) */
#define TF_ESTATE (-5)  /* call not valid in the object's current state */

/* Human-readable text of a status code (static storage). */
const char *tf_strerror(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int tf_version(void);

/* ------------------------------------------------------------------------
 * Elementwise twofold operations (Algorithms section of the paper).
 * z_i = x_i op y_i for i < n, each operand twofold (x0, x1) or dotted
 * (x1 == NULL).  z0 and z1 are required outputs of n elements.
 * ---------------------------------------------------------------------- */

/* Add: ATF1 for two twofolds, z0 = x0 + y0, z1 = (x1 + y1) + err(x0 + y0);
 * ATF1.1 when one operand is dotted (z1 = RN(dz0) exactly); the exact
 * Two-Sum (Algorithm 1.2) when both are dotted. */
int tf_add(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
           const void *y1, void *z0, void *z1, hipStream_t stream);

/* Subtract: STF1, z0 = x0 - y0, z1 = (x1 - y1) + err(x0 - y0); STF1.1 when y
 * is dotted; err(x0 - y0) - y1 when x is dotted; the exact Two-Diff
 * (Algorithm 2.2, with a - b = d + t) when both are dotted. */
int tf_sub(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
           const void *y1, void *z0, void *z1, hipStream_t stream);

/* Multiply: MTF1, z0 = x0 y0, z1 = (e00 + x1 y1) + (x0 y1 + x1 y0) with e00
 * the fma error of x0 y0; MTF1.1 when one operand is dotted; the exact
 * Two-Product (Algorithm 3) when both are dotted. */
int tf_mul(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
           const void *y1, void *z0, void *z1, hipStream_t stream);

/* Divide: DTF1, z0 = x0 / y0, r0 = fma(-z0, y0, x0), r1 = fma(-z0, y1, x1),
 * z1 = (r0 + r1) / (y0 + y1); DTF1.1 when y is dotted; DTF1.1.1 when both
 * are dotted (z1 = RN(dz0)); DTF1 with x1 = +0 when only x is dotted.
 * y0 == 0 gives infinite or NaN parts, as the IEEE operations do. */
int tf_div(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
           const void *y1, void *z0, void *z1, hipStream_t stream);

/* Square root: RTF1 for a twofold argument (z0 = sqrt(x0); renormalise x with
 * Two-Sum; one Newton step RPF1 on the renormalised pair; subtract z0 with
 * STF1.1 and add the two parts); RPF1.1 for a dotted argument,
 * z1 = fma(-z0, z0, x0) / (2 z0).  sqrt(0) gives z1 = NaN (0/0) and a
 * negative argument NaN parts, by the formulas themselves. */
int tf_sqrt(int dtype, int64_t n, const void *x0, const void *x1, void *z0, void *z1,
            hipStream_t stream);

/* ------------------------------------------------------------------------
 * Streaming kernels composed of the operations above.
 * ---------------------------------------------------------------------- */

/* axpy: z_i = a x_i + y_i with a twofold scalar a = (a[0], a[1]) (HOST
 * pointer to 2 values of dtype).  t = MTF1(a, x_i) (MTF1.1 if x is dotted),
 * z_i = ATF1(t, y_i) (ATF1.1 if y is dotted). */
int tf_axpy(int dtype, int64_t n, const void *a, const void *x0, const void *x1,
            const void *y0, const void *y1, void *z0, void *z1, hipStream_t stream);

/* Horner evaluation of p(x_i) = c[0] + c[1] x_i + ... + c[d] x_i^d with
 * dotted coefficients c (HOST pointer to degree + 1 values of dtype),
 * 0 <= degree <= TF_MAX_DEGREE: r = (c[d], +0); for k = d-1 .. 0,
 * r = ATF1.1(MTF1(r, x_i), c[k]) (MTF1.1 if x is dotted). */
#define TF_MAX_DEGREE 32
int tf_horner(int dtype, int64_t n, int degree, const void *c, const void *x0,
              const void *x1, void *z0, void *z1, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Reductions with a twofold accumulator over a fixed pairwise tree.
 *
 * Tree: the leaves (index order) are cut into tiles of 256 consecutive
 * indices, a short last tile padded with zero leaves; within a tile the
 * tree is complete with adjacent pairing (level 1 joins leaves 2i, 2i+1,
 * and so on for 8 levels); the tile results are joined by the same adjacent
 * pairing, their count padded with (+0, +0) to a power of two.  Every node
 * is ATF1(left, right); dotted leaves of tf_sum enter through Two-Sum at
 * level 1.  The tree depends only on n, never on the launch geometry, so
 * results are bitwise reproducible.
 *
 * out: DEVICE pointer to 2 values of dtype, written (z0, z1).
 * work / work_bytes: caller-owned device workspace of at least
 * tf_reduce_workspace_bytes(dtype, n) bytes (may be NULL when that is 0).
 * ---------------------------------------------------------------------- */
size_t tf_reduce_workspace_bytes(int dtype, int64_t n);

/* Sum of the twofold leaves (x0_i, x1_i), or of the dotted x0_i when x1 is
 * NULL. */
int tf_sum(int dtype, int64_t n, const void *x0, const void *x1, void *out, void *work,
           size_t work_bytes, hipStream_t stream);

/* Dot product: leaves are the twofold products of x_i and y_i, Two-Product
 * for dotted x and y (the paper's twofold accumulator of plain numbers),
 * MTF1 for twofold x and y, MTF1.1 for one twofold and one dotted. */
int tf_dot(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
           const void *y1, void *out, void *work, size_t work_bytes, hipStream_t stream);

/* tf_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels, tree and bits as tf_dot, with the partials kept in a
 * statically allocated device array of TF_NOALLOC_SCRATCH_BYTES instead of
 * a caller workspace.  Allocates nothing and calls no allocating routine;
 * the caller still owns x0, x1, y0, y1 and out (arguments as tf_dot).
 * Each GPU holds its own copy of the array, resident until the process
 * ends; its address is looked up on the first call on that device (the
 * device current at the call, which must be the stream's).  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other host threads) race and give undefined results; calls in
 * one stream are ordered and safe.  Nothing in the array needs to start at
 * zero: every partial is written before it is read.  When the partials of
 * n leaves at the current tiling would not fit, the call takes more tiles
 * per block (the tree, and so the result, does not depend on it); TF_ENOMEM
 * when even 256 tiles per block leave too many (n beyond about 2^34 in
 * binary64, 2^35 in binary32); TF_EINVAL as tf_dot; TF_EDEVICE when the
 * address lookup or a launch fails. */
#define TF_NOALLOC_SCRATCH_BYTES (4u << 20)
int tf_dot_noalloc(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
                   const void *y1, void *out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Plain (non-twofold) counterparts: the same kernels' standard results only
 * (z = the z0 the twofold call would produce, bit for bit), for measuring
 * the twofold/plain slowdown.  Arguments as above with single arrays.
 * ---------------------------------------------------------------------- */
int tf_plain_add(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream);
int tf_plain_sub(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream);
int tf_plain_mul(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream);
int tf_plain_div(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream);
int tf_plain_sqrt(int dtype, int64_t n, const void *x, void *z, hipStream_t stream);
/* z_i = a[0] x_i + y_i (a: HOST pointer to one value of dtype). */
int tf_plain_axpy(int dtype, int64_t n, const void *a, const void *x, const void *y, void *z,
                  hipStream_t stream);
/* r = c[d]; r = r x_i + c[k] for k = d-1 .. 0 (multiply, then add). */
int tf_plain_horner(int dtype, int64_t n, int degree, const void *c, const void *x, void *z,
                    hipStream_t stream);
/* Plain sums over the same tree (out: one value). */
int tf_plain_sum(int dtype, int64_t n, const void *x, void *out, void *work, size_t work_bytes,
                 hipStream_t stream);
int tf_plain_dot(int dtype, int64_t n, const void *x, const void *y, void *out, void *work,
                 size_t work_bytes, hipStream_t stream);

/* Memory roofline probe (the paper's vmem test): reads x and y, writes z = x,
 * n elements of dtype; moves the bytes of a plain binary operation with no
 * arithmetic. */
int tf_vmem(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Coupled ("p") algorithms and Dekker mode (Dekker arithmetic section;
 * Algorithms 1.1, MPF1, DPF1, RPF1).  A coupled twofold has |z1| at most
 * half an ulp of z0 (the result of a renormalisation); the p-algorithms
 * drop the terms that are negligible for such operands.
 * ---------------------------------------------------------------------- */

/* Operation codes of tf_coupled and tf_chain. */
#define TF_OP_ADD 0
#define TF_OP_SUB 1
#define TF_OP_MUL 2
#define TF_OP_DIV 3
#define TF_OP_SQRT 4

/* z_i = x_i op y_i with the coupled algorithm of op: ATF1 / STF1 for add and
 * subtract (the paper keeps the fast twofold algorithms for coupled input);
 * MPF1 for multiply, z1 = e00 + (x0 y1 + x1 y0) (x1 y1 dropped); DPF1 for
 * divide, z1 = (r0 + r1) / y0 (y1 not added to the divisor); RPF1 for the
 * square root (one Newton step on the pair, no renormalisation first).
 * Dotted operands give the same forms as the twofold calls (MPF1.1 is
 * MTF1.1, DPF1.1 is DTF1.1, RPF1.1 as tf_sqrt); a dotted dividend over a
 * twofold divisor is DPF1 with x1 = +0.  renorm != 0 passes every result
 * through Fast Two-Sum (Algorithm 1.1), the Dekker mode: the output is then
 * coupled and z0 is the rounded value of the pair, no longer the standard
 * result.  y0 / y1 are ignored for TF_OP_SQRT.  Other arguments as tf_add;
 * TF_EINVAL for an unknown op. */
int tf_coupled(int dtype, int op, int renorm, int64_t n, const void *x0, const void *x1,
               const void *y0, const void *y1, void *z0, void *z1, hipStream_t stream);

/* Renormalise twofolds with Fast Two-Sum (Algorithm 1.1):
 * s_i = z0_i + z1_i, t_i = z1_i - (s_i - z0_i); exact (s + t = z0 + z1) when
 * |z0_i| >= |z1_i|, computed literally otherwise.  z0, z1 required; s and t
 * may alias them exactly. */
int tf_renorm(int dtype, int64_t n, const void *z0, const void *z1, void *s, void *t,
              hipStream_t stream);

/* ------------------------------------------------------------------------
 * Chains: the compute-bound regime of the paper's performance criteria
 * (Introduction; Performance: the "10x" criterion for data already in
 * cache).  For each i the state starts at z = (x0_i, x1_i), or (x0_i, +0)
 * when x1 is NULL, and `reps` times z = z op y_i (TF_OP_SQRT: z = sqrt(z)),
 * the value staying in registers; y is dotted when y1 is NULL.
 *   mode TF_MODE_TWOFOLD  ATF1, STF1, MTF1, DTF1, RTF1 (and the *.1 forms for
 *                         a dotted y);
 *   mode TF_MODE_COUPLED  ATF1, STF1, MPF1, DPF1, RPF1;
 *   mode TF_MODE_DEKKER   the coupled step followed by Fast Two-Sum (the
 *                         paper's renormalising accumulator).
 * reps >= 0 (0 copies the start value).  HBM traffic is one read of each
 * input and one write of each output; the rest is arithmetic. */
#define TF_MODE_TWOFOLD 0
#define TF_MODE_COUPLED 1
#define TF_MODE_DEKKER 2
int tf_chain(int dtype, int op, int mode, int64_t n, int64_t reps, const void *x0, const void *x1,
             const void *y0, const void *y1, void *z0, void *z1, hipStream_t stream);

/* Plain chain: z_i = x_i, then reps times z_i = z_i op y_i (sqrt: sqrt(z_i)). */
int tf_plain_chain(int dtype, int op, int64_t n, int64_t reps, const void *x, const void *y, void *z,
                   hipStream_t stream);

/* ------------------------------------------------------------------------
 * Applications, batched (Applications section): many independent small
 * problems, one per GPU thread.
 * ---------------------------------------------------------------------- */

/* Back-substitution of nsys upper-triangular m x m systems U x = f
 * (Applications, Linear Ax=f; the paper's Jordan block is the bidiagonal
 * case), 1 <= m <= TF_MAX_TRSV: for i = m-1 down to 0, s = (f0, f1 or +0);
 * for j = i+1 .. m-1, s = STF1(s, MTF1(U_ij, x_j)); x_i = DTF1(s, U_ii).  A
 * NULL U1 makes the matrix dotted (MTF1.1 with U first, DTF1.1).  Entries
 * below the diagonal are never read.  Layout, k the system: U entry (i, j)
 * at [(i*m + j)*nsys + k]; f_i and x_i at [i*nsys + k].  x0 / x1 must not
 * overlap U or f. */
#define TF_MAX_TRSV 64
int tf_trsv_upper(int dtype, int64_t nsys, int m, const void *U0, const void *U1, const void *f0,
                  const void *f1, void *x0, void *x1, hipStream_t stream);
int tf_plain_trsv_upper(int dtype, int64_t nsys, int m, const void *U, const void *f, void *x,
                        hipStream_t stream);

/* Both roots of a_i x^2 + b_i x + c_i = 0 by the school formula
 * (Applications, Square root), every operand twofold (all six arrays
 * required): q = STF1(MTF1(b, b), MTF1(MTF1((4, 0), a), c)); d = RTF1(q);
 * e = MTF1((2, 0), a); r = DTF1(STF1(-b, d), e); s = DTF1(ATF1(-b, d), e).
 * A negative discriminant gives NaN in d and both roots; a zero one gives a
 * NaN error part (RTF1 at 0). */
int tf_quadratic(int dtype, int64_t n, const void *a0, const void *a1, const void *b0,
                 const void *b1, const void *c0, const void *c1, void *r0, void *r1, void *s0,
                 void *s1, hipStream_t stream);
int tf_plain_quadratic(int dtype, int64_t n, const void *a, const void *b, const void *c, void *r,
                       void *s, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Twofold fused multiply-add z_i = x_i y_i + w_i (an extension: the paper
 * defines + - * / and sqrt only).  z0 = fma(x0, y0, w0), bitwise the
 * hardware result; the error of that fma is rounded exactly with Boldo and
 * Muller's ErrFma steps (Two-Product of x0 y0, two Two-Sums); then
 * z1 = ((eps + x1 y1) + (x0 y1 + x1 y0)) + w1, the terms of an absent low
 * part left out.  x1, y1, w1 may each be NULL (dotted).
 * ---------------------------------------------------------------------- */
int tf_fma(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           const void *w0, const void *w1, void *z0, void *z1, hipStream_t stream);
int tf_plain_fma(int dtype, int64_t n, const void *x, const void *y, const void *w, void *z,
                 hipStream_t stream);

/* ------------------------------------------------------------------------
 * Launch tuning (process-wide).  Results never depend on these settings.
 *   TF_CFG_EW_BLOCKS_PER_CU    cap on the elementwise grid, in blocks per
 *                              compute unit (0 = one block per 256 threads'
 *                              worth of work, no cap; default 0)
 *   TF_CFG_RED_TILES_PER_BLOCK 256-leaf tiles per first-pass reduction
 *                              block, a power of two in [1, 256], or 0
 *                              (default) for the tuned value of each type
 *                              and leaf kind
 *   TF_CFG_RED_WAVES           waves per first-pass reduction block: 4, 8,
 *                              16, or 0 (default) for the tuned value
 * Returns the previous value, or TF_EINVAL for an unknown key or value.
 * ---------------------------------------------------------------------- */
#define TF_CFG_EW_BLOCKS_PER_CU 1
#define TF_CFG_RED_TILES_PER_BLOCK 2
#define TF_CFG_RED_WAVES 3
int64_t tf_config(int key, int64_t value);

/* ------------------------------------------------------------------------
 * Serving: verification jobs admitted continuously into one persistent
 * kernel.
 *
 * A job is one sum, dot, axpy or Horner evaluation (the streaming kernels
 * above) of its own length and type.  Jobs queue in arrival order and are
 * admitted while a slot (at most TFS_MAX_SLOTS in flight) and room in the
 * server's HBM pool (budget_bytes: the job's generated inputs, outputs and
 * partials) are free; the head of the queue waits otherwise.  An admitted
 * job's descriptor is published to the device job table, and the
 * persistent kernel's workers claim its 4096-element units alongside those
 * of every other job in flight, the job with the least work left first: a
 * job with generated inputs first runs units that write them, then its
 * compute units.  Reductions use the same fixed tree as tf_sum / tf_dot and
 * elementwise results are per element, so a job's result is bit for bit the
 * same alone or in any mix.
 *
 * Per job the server reports the result (sum / dot: z0, z1; axpy / Horner:
 * max |z0_i|, max |z1_i|, the number of elements with |z1_i| > thr |z0_i|,
 * and order-independent digests of z0 and z1) and a flag raised when the
 * twofold error estimate is large: |z1| > thr |z0| for sum / dot, max |z1_i|
 * > thr max |z0_i| for axpy / Horner, or any non-finite value; thr defaults
 * to 2^-20 (the paper's "daemon" that signals when z1 grows large against
 * z0, Motivation and Applications sections).
 * ---------------------------------------------------------------------- */
#define TFS_MAX_SLOTS 64
#define TFS_OP_SUM 0
#define TFS_OP_DOT 1
#define TFS_OP_AXPY 2
#define TFS_OP_HORNER 3
/* Job inputs: RANDOM and ILLCOND are generated on the device from the job
 * seed with a counter-based SplitMix64 stream (ILLCOND: axpy with
 * y ~ -a x, Horner of (x - 1)^8 near x = 1, both cancelling); PROVIDED
 * reads caller-owned device buffers x0, x1, y0, y1 (x1 / y1 NULL = dotted),
 * which must stay valid until the job completes. */
#define TFS_KIND_RANDOM 0
#define TFS_KIND_ILLCOND 1
#define TFS_KIND_PROVIDED 2

typedef struct {
    int op;        /* TFS_OP_* */
    int dtype;     /* TF_F32 / TF_F64 */
    int kind;      /* TFS_KIND_* */
    int degree;    /* Horner degree, 0 .. TF_MAX_DEGREE */
    int64_t n;     /* 1 .. 4096 * 16383 elements (16383 units of 4096) */
    uint64_t seed; /* input generator seed (RANDOM, ILLCOND) */
    double a[2];   /* axpy twofold scalar (rounded to dtype) */
    double c[TF_MAX_DEGREE + 1]; /* Horner coefficients (rounded to dtype) */
    double threshold;            /* flag threshold; 0 selects 2^-20 */
    const void *x0, *x1, *y0, *y1; /* PROVIDED inputs (device pointers) */
} tfs_job;

typedef struct {
    uint64_t id;
    int status;    /* TF_OK */
    int op, dtype, kind;
    int flag;      /* 1 when the error estimate is large (see above) */
    int64_t n;
    double z0, z1;                 /* sum / dot result, widened to binary64 */
    double max_abs_z0, max_abs_z1; /* axpy / Horner */
    uint64_t n_flagged;            /* axpy / Horner: elements over threshold */
    uint64_t nonfinite;            /* non-finite results */
    uint64_t hash_z0, hash_z1;     /* axpy / Horner: sum of bit patterns mod 2^64 */
    double t_arrive;  /* scheduled arrival (tfs_submit argument), tfs_clock() seconds */
    double t_submit;  /* when tfs_submit was called */
    double t_admit, t_publish, t_done; /* admitted, published to the device, completion seen */
    double queue_us;               /* slot opened on the device to its first unit claimed */
    double gen_us;                 /* generation of RANDOM / ILLCOND inputs on the device */
    double device_us;              /* compute units: inputs ready to the record written */
} tfs_result;

typedef struct {
    int64_t pending, in_flight, completed;
    uint64_t budget_bytes, resident_bytes, peak_resident_bytes;
    uint64_t admission_waits;      /* times the queue head waited for memory */
    int kernel_alive;
} tfs_stats;

typedef struct tfs_server tfs_server;

/* Create a server on `device` with an HBM pool of budget_bytes and at most
 * max_slots (1 .. TFS_MAX_SLOTS) jobs in flight; launches the persistent
 * kernel.  NULL on failure. */
tfs_server *tfs_create(int device, uint64_t budget_bytes, int max_slots);

/* Queue a job (thread-safe, non-blocking).  t_arrive: its arrival time on
 * tfs_clock() (<= 0: now).  TF_EINVAL for a malformed job, TF_ENOMEM for a
 * job larger than the whole budget. */
int tfs_submit(tfs_server *s, const tfs_job *job, double t_arrive, uint64_t *id);

/* Move up to `max` completed results into out[]; returns how many. */
int tfs_poll(tfs_server *s, tfs_result *out, int max);

/* Counters of the server (thread-safe). */
int tfs_get_stats(tfs_server *s, tfs_stats *out);

/* Seconds on the server clock (monotonic, process-wide). */
double tfs_clock(void);

/* Stop the server: jobs already published to the device run to
 * completion before the persistent kernel exits, queued jobs are dropped;
 * then free everything. */
int tfs_destroy(tfs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* TF_H */
