/*
 * hygt.h - batched Hypercube-Givens transforms (HyGT) on AMD Instinct MI355X
 * (gfx950).
 *
 * The transform is the one of Said, Zhao, Karczewicz, Egilmez, Seregin, Chen,
 * "Highly Efficient Non-Separable Transforms for Next Generation Video
 * Coding" (arXiv 2505.21728):
 *
 *   - A block is a vector of N = 2^log2n residuals (Sec. II: the residual
 *     vector r = x - p of one video block). A 2^B x 2^B pixel block is stored
 *     in row-major raster order (index = row * 2^B + col).
 *   - Each block carries a class index c (Sec. II: the classification index
 *     chosen per block); each class has its own angle set (Sec. III: one set
 *     of parameter vectors per class).
 *   - One pass rotates every index pair (i, i XOR 2^k) by its own angle with
 *     the Givens matrix of Sec. IV: y_m = cos*x_m + sin*x_n,
 *     y_n = -sin*x_m + cos*x_n, where m is the index of the pair whose bit k
 *     is 0 (the parallel-Givens matrix of eq. (8)).
 *   - A round is log2n passes, k = 0, 1, ..., log2n-1 (Sec. IV, hypercube
 *     dimensions taken in turn). The transform is R rounds; the first pass
 *     applied is round 0, pass 0 (the factor F_1 of eq. (5)).
 *   - Angle j of pass k belongs to the pair whose lower index m is j with a
 *     zero bit inserted at bit position k, upper index n = m + 2^k (the index
 *     arrays of Fig. 5). There are R * N * log2n / 2 angles per class (Sec. IV).
 *   - The inverse applies the passes in reverse order with negated angles
 *     (eq. (6), eq. (9), Sec. IV); it equals the transpose.
 *   - The optional final permutation pass of Fig. 4 is applied only by
 *     hygt_apply_perm(); the other entry points leave it out.
 *
 * Memory and ownership
 *   Every array argument is DEVICE memory owned by the caller. The library
 *   allocates nothing, keeps no state between calls (apart from the static
 *   area of hygt_transform_noalloc()) and never synchronises the stream
 *   except in hygt_check_error(). All work is enqueued on `stream` (0 = the
 *   null stream) and runs asynchronously.
 *
 * Layouts
 *   x, y     float32 [nblocks][N], contiguous, 16-byte aligned.
 *            y == x (in place) is allowed; any other overlap is rejected.
 *   cls      int32 [nblocks], class of each block in [0, nclasses).
 *            May be NULL when nclasses == 1 (every block is class 0).
 *   Any array pointer may be NULL when nblocks == 0.
 *   angles   float32 [nclasses][rounds][log2n][N/2], contiguous, radians.
 *   workspace  at least hygt_workspace_bytes(...) bytes, 256-byte aligned.
 *            Holds the class grouping and the per-class multiplier tables
 *            built by hygt_plan(); it needs no initialisation. Calls that
 *            use one workspace must be ordered (one stream, or events).
 *
 * Limits
 *   1 <= log2n <= 8, 1 <= rounds <= HYGT_MAX_ROUNDS,
 *   1 <= nclasses <= HYGT_MAX_CLASSES, 0 <= nblocks <= HYGT_MAX_BLOCKS.
 *   Inputs are expected to be finite with Euclidean block norm below 2^90;
 *   within that range every output is within a few FP32 ulps per pass of the
 *   exact transform (relative L2 well under 1e-5 for the sizes above).
 *
 * Errors
 *   Every entry point returns a status. Host-side validation failures return
 *   HYGT_EINVAL or HYGT_EWORKSPACE and enqueue nothing. nblocks == 0 is a
 *   successful no-op. A class index outside [0, nclasses) is detected on the
 *   device: that block is left unwritten and a flag is set in the workspace,
 *   which hygt_check_error() reports as HYGT_ECLASS.
 *
 * Determinism
 *   Each block's result depends only on that block's values, its class and
 *   the angle table: it is bit-identical whatever the batch it is in, the
 *   batch order, or in-place versus out-of-place execution. The one
 *   exception is hygt_backward()'s per-class angle gradient, a sum of FP32
 *   atomic additions whose order, and so whose last bits, vary.
 */
#ifndef HYGT_H
#define HYGT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hygt_status {
    HYGT_OK = 0,
    HYGT_EINVAL = -1,     /* an argument is out of range, NULL or misaligned */
    HYGT_EWORKSPACE = -2, /* workspace NULL, too small or not 256-byte aligned */
    HYGT_ELAUNCH = -3,    /* the HIP runtime refused a kernel launch */
    HYGT_ECLASS = -4,     /* a block's class index was outside [0, nclasses) */
    HYGT_EHIP = -5,       /* another HIP runtime error (hygt_check_error) */
    HYGT_ESCRATCH = -6    /* the sizes need more than the static scratch area
                             of hygt_transform_noalloc() */
};

enum hygt_direction {
    HYGT_FORWARD = 0, /* y = T_c x   (eq. (5)) */
    HYGT_INVERSE = 1  /* y = T_c^-1 x = T_c^T x   (eq. (6), eq. (9)) */
};

#define HYGT_MAX_LOG2N 8
#define HYGT_MAX_ROUNDS 64
#define HYGT_MAX_CLASSES 4096
#define HYGT_MAX_BLOCKS 2147483647LL

/* Size in bytes of the workspace needed for these sizes (0 for invalid
 * sizes). The same workspace serves hygt_plan, hygt_apply, hygt_forward and
 * hygt_inverse for these sizes. */
size_t hygt_workspace_bytes(int64_t nblocks, int log2n, int rounds, int nclasses);

/* Builds, in the workspace, everything that depends on the classes and the
 * angles but not on the data (two kernel launches):
 *   - the multiplier tables of both directions: every angle converted in
 *     FP64 into per-pass FP32 multipliers (Sec. IV and Fig. 6 store
 *     compact parameters and expand them into wider multipliers at use):
 *     the two multipliers of a three-step lifting form of each
 *     rotation, or for N = 256 and the passes along bit 7, its cosine and
 *     sine;
 *   - the blocks sorted by class over the whole batch into tiles of 64
 *     blocks of one class (a counting sort), with a flag for any class
 *     index outside [0, nclasses).
 * cls is read; angles is read. Both may be reused or freed once the stream
 * reaches the end of this call's work. */
int hygt_plan(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
              const float* angles, int nclasses,
              void* workspace, size_t workspace_bytes, hipStream_t stream);

/* hygt_plan() with the parameters given as 8-bit codes (Fig. 6: one byte per
 * parameter, converted to multipliers only when needed; the paper does not
 * give the code-to-angle map): code q stands for the angle
 * (q - 128) * pi / 128, so 256 codes cover [-pi, pi) in equal steps and
 * q = 128 is the zero angle. codes: uint8 [nclasses][rounds][log2n][N/2].
 * The multipliers are computed from the exact angle in FP64, so a plan from
 * codes equals a plan from the FP32 angles closest to those angles only to
 * within the FP32 rounding of the angle. */
int hygt_plan_codes(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                    const uint8_t* codes, int nclasses,
                    void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Applies the planned transform (direction HYGT_FORWARD or HYGT_INVERSE) to
 * x, writing y. The sizes must be those given to the hygt_plan() call that
 * filled the workspace; the plan may be applied any number of times, in both
 * directions, until the workspace is planned again. */
int hygt_apply(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
               int nclasses, int direction,
               const void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Largest block length (log2) of hygt_apply_perm(). */
#define HYGT_PERM_MAX_LOG2N 6

/* hygt_apply() with the optional final permutation pass of Fig. 4, which
 * orders each class's coefficients (by variance, in the paper):
 *   forward:  y[b][i] = (T_c x[b])[perm[c][i]];
 *   inverse:  undoes that permutation, then applies T_c^T.
 * perm: int32 [nclasses][N], each row a permutation of 0..N-1 (device
 * memory; entries are used modulo N, so a bad row gives wrong results, never
 * an access outside the block). 2 <= log2n <= HYGT_PERM_MAX_LOG2N. */
int hygt_apply_perm(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                    int nclasses, int direction, const int32_t* perm,
                    const void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Largest block length (log2) of the integer transform. */
#define HYGT_INT_MAX_LOG2N 6

/* Plan for the integer transform (Sec. IV, Fig. 6: one byte per parameter,
 * converted through a shared table of sines and cosines into higher
 * precision multipliers; integer arithmetic as video coding standards need).
 * codes: uint8 [nclasses][rounds][log2n][N/2] in the layout of hygt_plan's
 * angles, code q meaning the angle (q - 128) pi / 128. Each pair gets the
 * fixed-point multipliers C = round(2^14 cos), S = round(2^14 sin) (FP64,
 * ties to even). 2 <= log2n <= HYGT_INT_MAX_LOG2N. The workspace is then for
 * hygt_apply_int() only. Other arguments and errors as hygt_plan(). */
int hygt_plan_int(const int32_t* cls, int64_t nblocks, int log2n, int rounds,
                  const uint8_t* codes, int nclasses, void* workspace,
                  size_t workspace_bytes, hipStream_t stream);

/* The integer transform of int32 blocks x[nblocks][N] into y (same layout;
 * y == x allowed, other overlaps rejected; 16-byte aligned). Every butterfly
 * of eq. (7) computes
 *   y_m = (C x_m + S x_n + 2^13) >> 14,   y_n = (C x_n - S x_m + 2^13) >> 14
 * (arithmetic shift: rounding to nearest, ties upwards). The inverse runs the
 * passes in reverse order with multipliers (C, -S) (eq. (9)); it undoes the
 * forward transform up to the rounding of each butterfly, not exactly.
 * Results are exact (bit-identical to this definition in unbounded integers)
 * for blocks of L2 norm at most 2^15, e.g. residuals within +-4095 for
 * N = 64; beyond that they are deterministic but unspecified. The workspace
 * must come from hygt_plan_int() with the same sizes. */
int hygt_apply_int(const int32_t* x, int32_t* y, int64_t nblocks, int log2n, int rounds,
                   int nclasses, int direction, const void* workspace,
                   size_t workspace_bytes, hipStream_t stream);

/* hygt_plan() followed by hygt_apply(HYGT_FORWARD): y[b] = T_{cls[b]} x[b]. */
int hygt_forward(const float* x, float* y, const int32_t* cls, int64_t nblocks,
                 int log2n, int rounds, const float* angles, int nclasses,
                 void* workspace, size_t workspace_bytes, hipStream_t stream);

/* hygt_plan() followed by hygt_apply(HYGT_INVERSE): y[b] = T_{cls[b]}^T x[b]. */
int hygt_inverse(const float* x, float* y, const int32_t* cls, int64_t nblocks,
                 int log2n, int rounds, const float* angles, int nclasses,
                 void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- For callers that cannot allocate ------------------------------------
 *
 * For code that may not call hipMalloc or take memory from an allocator (for
 * instance work captured into a HIP graph, or a serving loop that allocates
 * nothing per call): hygt_forward() (direction HYGT_FORWARD) or hygt_inverse()
 * (HYGT_INVERSE) with the workspace taken from a static device array of the
 * library, HYGT_NOALLOC_SCRATCH_BYTES bytes per GPU, held by each GPU the
 * library runs on until the process ends. The caller still passes x, y, cls
 * and angles (device memory, as for hygt_forward()). The call allocates
 * nothing; sizes whose workspace (hygt_workspace_bytes()) exceeds the area
 * are rejected with HYGT_ESCRATCH before anything is enqueued (for N = 64,
 * R = 4 and 35 classes: up to about 3.9 million blocks). Nothing in the area
 * needs clearing between calls: every call rewrites what it reads.
 *
 * All calls on one GPU share that GPU's area, so calls that may overlap on
 * the device (other streams, or other host threads) race and give wrong
 * results; order them (one stream, or events). hygt_check_error() cannot be
 * used for these calls (the area is not visible to the caller); class
 * indices must be in range. The first call on a device looks up the area's
 * device address (that call is not capturable; later ones are). */
#define HYGT_NOALLOC_SCRATCH_BYTES 16777216 /* 16 MiB */

int hygt_transform_noalloc(const float* x, float* y, const int32_t* cls, int64_t nblocks,
                           int log2n, int rounds, const float* angles, int nclasses,
                           int direction, hipStream_t stream);

/* Largest block length (log2) supported by hygt_backward(). */
#define HYGT_BACKWARD_MAX_LOG2N 6

/* Reverse-mode derivative of hygt_apply(HYGT_FORWARD), for the parameter
 * optimisation of Sec. V (a gradient step on the angles): given the forward
 * outputs y = T_c x and gy = dL/dy, writes
 *   gx       dL/dx = T_c^T gy for every block   [nblocks][N] float32;
 *   gangles  dL/dangles, summed over the blocks of each class
 *            [nclasses][rounds][log2n][N/2] float32 (same layout as angles,
 *            overwritten; classes without blocks get zeros).
 * Nothing from the forward call is needed but y: each pass's inputs are
 * recovered from its outputs by the inverse rotation (eq. (9)). For one
 * rotation, dL/dtheta = g_m y_n - g_n y_m. The workspace must hold a plan
 * (hygt_plan()) for these sizes and classes; its block grouping is used, and
 * this call builds its own inverse-direction multiplier table from `angles`
 * in a separate part of the workspace, so it must not overlap other
 * hygt_backward() calls on the same workspace. Alignment as for hygt_apply(); gx may be gy (in place) but not
 * y. log2n <= HYGT_BACKWARD_MAX_LOG2N. The per-class sums are FP32 atomic
 * additions, so their last bits can differ from run to run. */
int hygt_backward(const float* y, const float* gy, float* gx, float* gangles, int64_t nblocks,
                  int log2n, int rounds, const float* angles, int nclasses,
                  void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Block length (log2) supported by hygt_dense_apply(). */
#define HYGT_DENSE_LOG2N 6

/* The matrix-based transform that HyGT replaces, for comparison: the dense
 * per-class transform y[b] = M_{cls[b]} x[b] of eq. (3) (a KLT when M_c holds
 * the eigenvectors of the class's covariance, Sec. II), whose cost Table I
 * gives as N^2 operations and N^2 stored values per class. Runs on the
 * matrix cores as a grouped GEMM over the class-sorted tiles of the plan in
 * the workspace (only its class grouping is used, so the sizes must be
 * those of that hygt_plan() call).
 *   mats   BF16 bit patterns [nclasses][N][N], row-major (mats[c][i][j] is
 *          M_c[i][j]), 16-byte aligned; read only.
 *   x, y   as for hygt_apply(); N must be 64 (log2n == HYGT_DENSE_LOG2N).
 * Each x value is rounded to BF16 (to nearest, ties to even) before the
 * products, which are summed in FP32 (exact for integer residuals of at most
 * 8 significant bits, such as the [-255, 255] range of 8-bit video). Blocks
 * whose class was out of range are left unwritten. For T_c^T (the inverse of
 * an orthogonal T_c) pass the transposed matrices. */
int hygt_dense_apply(const float* x, float* y, int64_t nblocks, int log2n, int rounds,
                     int nclasses, const uint16_t* mats,
                     const void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- Mixed batches: several block sizes in one launch -------------------
 *
 * A codec transforms blocks of several sizes at once (Sec. VI uses 4x4 and
 * 8x8 transforms side by side). A mixed batch is a list of segments, one per
 * block size, each with its own blocks, classes and angle set; one
 * persistent launch transforms the tiles of all segments. */

#define HYGT_MAX_SEGMENTS 4

typedef struct hygt_segment {
    const float* x;       /* [nblocks][N] input, device memory */
    float* y;             /* [nblocks][N] output; may be x, must not overlap another segment */
    const int32_t* cls;   /* [nblocks] classes in [0, nclasses); NULL when nclasses == 1 */
    const float* angles;  /* [nclasses][rounds][log2n][N/2] */
    int64_t nblocks;
    int log2n;            /* 2 .. 8 (N = 4 .. 256) */
    int rounds;
    int nclasses;
    int reserved;         /* 0 */
} hygt_segment;

/* Workspace bytes for a mixed batch (0 if a segment is invalid). */
size_t hygt_mixed_workspace_bytes(const hygt_segment* segs, int nseg);

/* hygt_plan() of every segment, into consecutive parts of one workspace. */
int hygt_mixed_plan(const hygt_segment* segs, int nseg, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/* hygt_mixed_plan() without the multiplier tables: only the class grouping
 * of every segment, for callers whose angles have not changed since the
 * last hygt_mixed_plan() on this workspace with the same segment sizes
 * (nblocks, log2n, rounds, nclasses of every segment, which fix where each
 * segment's tables sit in the workspace; the classes and the x and y
 * buffers may change). The tables of that plan stay in the workspace and
 * are used as they are; with other angles or sizes, or on a workspace that
 * never held such a plan, the transform uses whatever the workspace holds.
 * A training step that changes the angles plans again with
 * hygt_mixed_plan(). */
int hygt_mixed_regroup(const hygt_segment* segs, int nseg, void* workspace,
                       size_t workspace_bytes, hipStream_t stream);

/* Number of launch configurations of hygt_mixed_apply(). */
int hygt_mixed_num_configs(void);

/* One launch of the mixed kernel over all segments, forward or inverse.
 * `config` in [0, hygt_mixed_num_configs()) picks the launch shape (grid size
 * and whether rounds are unrolled); hygt_mixed_autotune() finds the fastest.
 * The segments must be those of the hygt_mixed_plan() call that filled the
 * workspace. */
int hygt_mixed_apply(const hygt_segment* segs, int nseg, int direction, int config,
                     const void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Times every configuration of hygt_mixed_apply() on these segments (each
 * run once to warm up, then three times) and returns the fastest in
 * *best_config and its mean time in microseconds in *best_us. Synchronises
 * `stream`; writes the segments' outputs. */
int hygt_mixed_autotune(const hygt_segment* segs, int nseg, int direction,
                        const void* workspace, size_t workspace_bytes, hipStream_t stream,
                        int* best_config, float* best_us);

/* A captured HIP graph of hygt_mixed_plan() + hygt_mixed_apply() for fixed
 * buffers: replaying it re-plans and transforms whatever the buffers hold.
 * Created by stream capture on `capture_stream` (not the null stream); the
 * handle is a host object owned by the caller. */
typedef struct hygt_graph_s* hygt_graph;
int hygt_mixed_graph_create(const hygt_segment* segs, int nseg, int direction, int config,
                            void* workspace, size_t workspace_bytes, hipStream_t capture_stream,
                            hygt_graph* graph);
int hygt_graph_launch(hygt_graph graph, hipStream_t stream);
int hygt_graph_destroy(hygt_graph graph);

/* ---- Request queue: single-launch batches of requests (serving) ---------
 *
 * For a serving loop that transforms requests as they arrive (a codec's
 * frames, Sec. VI: blocks of one size each, with a class per block), where
 * latency rather than bulk throughput matters. The multiplier tables of each
 * block size are built once (hygt_table_build()) and stay on the device. The
 * requests themselves are descriptors in a ring in pinned host memory that
 * the caller fills: one launch (hygt_requests_apply()) transforms a run of
 * consecutive ring entries, with no plan, no workspace and no class grouping.
 * The call hands the run's descriptors to the launch with its arguments (so
 * that no wavefront reads host memory: such reads cost about 0.1 us each,
 * one after another, which for a launch of 512 workgroups took 1.3 ms), and
 * the device writes each request's status back into its ring entry.
 * A wavefront takes one block (N >= 64, N/64 values per lane) or 64/N
 * consecutive blocks (N <= 32, a value per lane), and a block's lanes read
 * its own class's table a pass at a time, exchanging values with lane
 * shuffles. A block's arithmetic, and so its result, is bit for bit that of
 * hygt_apply() with a plan of the same angles. Bulk batches are faster through hygt_plan() + hygt_apply(), whose
 * class-sorted tiles read each multiplier once per 64 blocks. */

/* Bytes of the table of one block size (0 for invalid sizes). */
size_t hygt_table_bytes(int log2n, int rounds, int nclasses);

/* Builds the multiplier tables of both directions (the same FP64 conversion
 * and sign bookkeeping as hygt_plan()) into `table`: device memory of at
 * least hygt_table_bytes() bytes, 256-byte aligned, owned by the caller and
 * read by every hygt_requests_apply() that names it. angles: device memory,
 * [nclasses][rounds][log2n][N/2] float32, read only; 2 <= log2n <= 8. One
 * launch of 2 * nclasses workgroups on `stream`. */
int hygt_table_build(const float* angles, int log2n, int rounds, int nclasses, void* table,
                     size_t table_bytes, hipStream_t stream);

/* A table built by hygt_table_build(), with its sizes. */
typedef struct hygt_table_ref {
    const void* table;
    int32_t log2n;
    int32_t rounds;
    int32_t nclasses;
    int32_t reserved; /* 0 */
} hygt_table_ref;

/* One request: nblocks blocks of one size. */
typedef struct hygt_request {
    const float* x;      /* [nblocks][N] input, device memory, 16-byte aligned */
    float* y;            /* [nblocks][N] output; may be x, must not overlap it otherwise */
    const int32_t* cls;  /* [nblocks] classes; NULL when the table has one class */
    int64_t nblocks;     /* 0 .. HYGT_MAX_REQUEST_BLOCKS */
    int32_t table;       /* index into the `tables` of the call */
    int32_t status;      /* written by the device: set to HYGT_ECLASS when some block's
                            class is outside [0, nclasses); the caller clears it */
    int64_t first_wg;    /* written by hygt_requests_apply(): the request's first
                            workgroup in its launch */
} hygt_request;

#define HYGT_MAX_BATCH_REQUESTS 64
#define HYGT_MAX_TABLES 4
#define HYGT_MAX_REQUEST_BLOCKS (1LL << 26)

/* Transforms requests ring[(first + i) % capacity], i = 0 .. count - 1
 * (1 <= count <= HYGT_MAX_BATCH_REQUESTS), forward or inverse, in one launch
 * on `stream`.
 *   ring    capacity entries in pinned host memory that the device can
 *           write (hipHostMalloc), 8-byte aligned; other memory is rejected
 *           with HYGT_EINVAL (hipHostGetDevicePointer gives the device's
 *           address of the ring). The host part of this call reads the
 *           entries (they may be rewritten as soon as it returns) and writes
 *           their first_wg; the device writes the status of a request with a
 *           class out of range, so the statuses are final once the stream
 *           has passed the end of this call's work.
 *   tables  ntables (1 .. HYGT_MAX_TABLES) table references, host memory,
 *           read during the call; the tables themselves must stay until
 *           the work ends.
 * A block whose class is out of range is written as zeros (never left
 * with stale contents) and sets its request's status. Requests with no
 * blocks are skipped. Entry checks (sizes, table index, NULL or misaligned
 * pointers, partial overlap of x and y) run on the host before anything is
 * enqueued: a failing entry makes the call return HYGT_EINVAL with nothing
 * launched. Different requests must not write overlapping outputs. */
int hygt_requests_apply(hygt_request* ring, int64_t capacity, int64_t first, int count,
                        const hygt_table_ref* tables, int ntables, int direction,
                        hipStream_t stream);

/* Waits for `stream`, then reports whether the last non-empty plan on this
 * workspace met a class index outside [0, nclasses) (HYGT_ECLASS), a HIP
 * error (HYGT_EHIP), or neither (HYGT_OK). Reads at most workspace_bytes
 * bytes of the workspace. A plan of zero blocks launches nothing and writes
 * nothing, so on a workspace (or a mixed batch's part) that has only seen
 * such plans the answer is undefined: there is nothing to check, and the
 * caller should not ask (the Python binding skips those parts). */
int hygt_check_error(const void* workspace, size_t workspace_bytes, hipStream_t stream);

/* A static, human-readable description of a status code. */
const char* hygt_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* HYGT_H */
