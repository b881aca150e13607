/*
 * dpd.h -- C ABI of libdpd, an MI355X (gfx950) implementation of the
 * augmented parallel Hammerstein (APH) digital predistorter of Li et al.,
 * "Parallel Digital Predistortion Design on Mobile GPU and Embedded Multicore
 * CPU for Mobile Transmitters".
 *
 * What the library computes (Eq. 1, section 2.1; Algorithm 1, section 3):
 *
 *   z_n = c + sum_{p in I_P} sum_{k=0}^{L-1} h_{p,k} psi_p(x_{n-k})
 *           + sum_{q in I_Q} sum_{k=0}^{L-1} hbar_{q,k} conj(psi_q(x_{n-k})),
 *   psi_p(x) = |x|^(p-1) x     (odd orders p, monomial basis),
 *
 * for n = 0..N-1, with x_m = 0 for m < 0 unless a history is carried.  The tap
 * sum has L terms (k = 0..L-1), matching the L-entry coefficient vectors of
 * section 2.2.  Arithmetic is IEEE FP32 with fused multiply-add.
 *
 * Conventions shared by every entry point
 *   - Samples are interleaved complex64 (float re, float im; 8 bytes), in
 *     device memory owned by the caller.  Pointers must be 8-byte aligned;
 *     16-byte alignment (and an even row stride) selects the vector fast path.
 *   - Coefficients use the stacking of section 2.2: for each main-branch order
 *     (in the order passed to dpd_create) its L taps, then for each
 *     conjugate-branch order its L taps, then c.  K = (n_main + n_conj)*L + 1
 *     complex values, interleaved as 2K floats.
 *   - Orders are odd, 1 <= p <= 15, strictly ascending within a branch; the
 *     same order may appear in both branches.  1 <= L <= 16.
 *   - A stream argument is a hipStream_t passed as void* (NULL = the null
 *     stream).  Device work is enqueued asynchronously on it; no call below
 *     synchronizes the host unless it says so.
 *   - Every call returns a dpd_status.  Nothing throws or aborts across the
 *     ABI; out-parameters are left untouched on failure.  DPD_EHIP carries the
 *     HIP error code in dpd_last_hip_error() (per host thread).  Kernel faults
 *     surface at the caller's next synchronization.
 *   - Input and output ranges must not overlap (later tiles read halo samples
 *     that earlier tiles would already have overwritten): overlap is
 *     DPD_EINVAL.
 */
#ifndef DPD_H
#define DPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dpd_status {
    DPD_OK = 0,
    DPD_EINVAL = 1,        /* bad argument, null pointer, overlap, misalignment */
    DPD_EUNSUPPORTED = 2,  /* order > 15, L > 16, or a size beyond the limits  */
    DPD_ENOMEM = 3,        /* device or host allocation failed                 */
    DPD_EHIP = 4           /* a HIP runtime call failed (dpd_last_hip_error)   */
} dpd_status;

typedef struct dpd_plan dpd_plan;
typedef struct dpd_batch dpd_batch;

/* Launch shape of the forward kernels; chosen by the autotuner or defaulted.
 *   samples_per_thread: consecutive outputs per thread (2, 4 or 8)
 *   stage_lds: 1 = the tile and its (L-1)-sample halo are staged through LDS
 *              with coalesced 16-byte loads, 0 = each thread loads its own
 *              window (halo re-reads hit the cache)
 *   block: threads per block (must be 256; other values are rejected)
 *   grid_mult: persistent batched kernel only -- resident blocks per CU */
typedef struct dpd_tune {
    int32_t samples_per_thread;
    int32_t stage_lds;
    int32_t block;
    int32_t grid_mult;
} dpd_tune;

/* ------------------------------------------------------------------ plans --
 * dpd_create -- validate the order sets and L, copy the K host coefficients,
 * precombine them into the device table the kernels read, and return a plan
 * (section 2.1 basis and filters; section 2.2 coefficient stacking).
 *   main_orders[n_main]  odd orders of the main branch, n_main >= 1
 *   conj_orders[n_conj]  odd orders of the conjugate branch, n_conj >= 0
 *                        (NULL allowed when n_conj == 0)
 *   L                    taps per filter, 1..16
 *   coeffs_host          2K floats (host memory), section 2.2 layout
 *   out                  receives the plan; the caller frees it with
 *                        dpd_destroy.  The plan owns its device table.
 * Synchronous (device allocation + copy).  Uses the current HIP device. */
dpd_status dpd_create(const int32_t *main_orders, int32_t n_main,
                      const int32_t *conj_orders, int32_t n_conj, int32_t L,
                      const float *coeffs_host, dpd_plan **out);

/* dpd_destroy -- frees the plan.  Freeing device memory waits for the device
 * (work on every stream that may still read the plan's table), so destroy
 * plans outside latency-critical loops.  NULL is a no-op. */
dpd_status dpd_destroy(dpd_plan *plan);

/* dpd_num_coeffs -- K, the number of complex coefficients of the plan. */
dpd_status dpd_num_coeffs(const dpd_plan *plan, int32_t *K);

/* dpd_set_coeffs -- replace the coefficients from host memory (2K floats).
 * Not tied to a stream, so it waits for the device (every stream) before
 * overwriting the table: each call enqueued before it uses the old
 * coefficients, each call after it the new ones.  In loops use
 * dpd_set_coeffs_async or dpd_set_coeffs_device.
 *
 * dpd_set_coeffs_async -- the same update ordered on `stream` (NULL: the null
 * stream): work enqueued on that stream before it sees the old coefficients,
 * work after it the new ones; work on other streams that uses the plan is
 * the caller's to order (events).  The host copies the table into a pinned
 * staging buffer of the plan (allocated on the first call) and waits only for
 * the previous copy out of that buffer; coeffs_host may be reused on return.
 * Calls on one plan from several host threads must be serialized by the
 * caller. */
dpd_status dpd_set_coeffs(dpd_plan *plan, const float *coeffs_host);
dpd_status dpd_set_coeffs_async(dpd_plan *plan, const float *coeffs_host, void *stream);

/* dpd_set_coeffs_device -- replace the coefficients from device memory
 * (K complex64), stream-ordered on `stream` with no host synchronization.
 * Work on other streams that uses this plan must be ordered by the caller. */
dpd_status dpd_set_coeffs_device(dpd_plan *plan, const void *coeffs_dev, void *stream);

/* dpd_set_coeffs_device_if -- as dpd_set_coeffs_device, but only when the
 * device int32 *flag_dev is 0 when the copy runs (stream order); otherwise
 * the plan keeps its coefficients.  With the info output of dpd_ls_solve as
 * the flag, a failed solve (NaN coefficients) never reaches the plan, without
 * a host round trip.  flag_dev: device, 4-byte aligned, read only. */
dpd_status dpd_set_coeffs_device_if(dpd_plan *plan, const void *coeffs_dev, const int32_t *flag_dev,
                                    void *stream);

/* dpd_set_tune / dpd_get_tune -- launch shape of this plan's forward kernels.
 * Fields outside the supported set are DPD_EINVAL. */
dpd_status dpd_set_tune(dpd_plan *plan, const dpd_tune *tune);
dpd_status dpd_get_tune(const dpd_plan *plan, dpd_tune *tune);

/* ---------------------------------------------------------------- forward --
 * dpd_apply -- Eq. (1) / Algorithm 1 on one stream of n samples with zero
 * pre-history: out[t] = z_t for t = 0..n-1.  in, out: device complex64 (device
 * memory, or the device mapping of pinned host memory from
 * hipHostGetDevicePointer: the zero-copy form of section 3.3.1, where the
 * kernel reads and writes across the host link).
 * n == 0 is a no-op returning DPD_OK. */
dpd_status dpd_apply(dpd_plan *plan, void *stream, const void *in, void *out, int64_t n);

/* dpd_apply_rows -- `rows` independent streams of n samples sharing the plan;
 * row r starts at in + r*ld and out + r*ld (ld in samples, ld >= n).  The
 * filter memory never crosses a row: every row starts from zero history. */
dpd_status dpd_apply_rows(dpd_plan *plan, void *stream, const void *in, void *out,
                          int64_t rows, int64_t n, int64_t ld);

/* dpd_apply_coeffs -- as dpd_apply_rows, but the coefficients are read from a
 * device array of K complex64 (section 2.2 layout) in stream order, without a
 * host round trip (used by training).  They are precombined into a second
 * table of the plan, used only by calls that pass device coefficients (this
 * one and dpd_backward with coeffs_dev): the plan's own coefficients stay as
 * they were.  Such calls on one plan that overlap in time (different
 * streams) race on that second table; order them, or use one plan each. */
dpd_status dpd_apply_coeffs(dpd_plan *plan, void *stream, const void *coeffs_dev,
                            const void *in, void *out, int64_t rows, int64_t n, int64_t ld);

/* dpd_apply_hist -- streaming form: `hist` (device, L-1 complex64, oldest
 * first) holds the inputs that precede in[0]; it is read, then overwritten
 * with the last L-1 inputs of hist ++ in.  Calling it on consecutive chunks
 * gives the same outputs as one call on the whole stream (the zero-filled
 * pre-history of Eq. 2 is the special case hist = 0).  hist may be NULL only
 * when L == 1. */
dpd_status dpd_apply_hist(dpd_plan *plan, void *stream, const void *in, void *out, int64_t n,
                          void *hist);

/* --------------------------------------------------------------- backward --
 * Gradient of a real loss E through Eq. (1) (not in the paper).  Complex
 * gradients follow the convention dE/dRe + j dE/dIm (the one PyTorch uses).
 *   coeffs_dev   K complex64 on the device, or NULL to use the plan's (device
 *                coefficients go through the plan's second table, as in
 *                dpd_apply_coeffs; the plan's own coefficients are untouched;
 *                read only when grad_x is requested: dE/dcoeffs does not
 *                depend on the coefficients)
 *   x            inputs of the forward call, rows x n with row stride ld
 *   grad_z       dE/dz for the outputs, same shape
 *   grad_x       receives dE/dx (same shape), or NULL to skip it
 *   grad_coeffs  receives dE/dcoeffs (K complex64, summed over all rows), or
 *                NULL to skip it
 *   ws, ws_bytes device workspace of at least dpd_backward_ws_size() bytes
 * Deterministic: the same inputs give bitwise the same gradients.  Rows start
 * from zero history.  dE/dcoeffs is summed in FP32 over at most 128 samples
 * per lane, then in FP64, so its accuracy does not degrade with rows * n (any
 * size that fits in memory, 64-bit indices throughout). */
dpd_status dpd_backward_ws_size(const dpd_plan *plan, int64_t rows, int64_t n, size_t *bytes);
dpd_status dpd_backward(dpd_plan *plan, void *stream, const void *coeffs_dev, const void *x,
                        const void *grad_z, void *grad_x, void *grad_coeffs, int64_t rows,
                        int64_t n, int64_t ld, void *ws, size_t ws_bytes);

/* dpd_backward_noalloc -- for callers that cannot allocate device memory or
 * pass a workspace (code under stream capture into a graph, tight serving
 * loops, harnesses that forbid allocation): dpd_backward with the same
 * arguments minus the workspace, the same kernels and bitwise the same
 * results.  The per-block partial sums of the coefficient gradient live in a
 * fixed device array of the library (4.25 MiB per GPU, held until the process
 * ends); a plan whose partials need more (only on devices with many more
 * compute units than the MI355X's 256) is DPD_EUNSUPPORTED.  It calls no
 * allocator.  The array is shared by every call on one GPU: calls with a
 * coefficient gradient that overlap in time on one GPU (different streams or
 * host threads) race on it -- order them.  Calls without grad_coeffs use no
 * scratch. */
dpd_status dpd_backward_noalloc(dpd_plan *plan, void *stream, const void *coeffs_dev, const void *x,
                                const void *grad_z, void *grad_x, void *grad_coeffs, int64_t rows,
                                int64_t n, int64_t ld);

/* ---------------------------------------------------------------- batched --
 * Many streams of uneven length, each with its own order set, L and
 * coefficients, in one persistent launch (many antennas of a massive-MIMO
 * transmitter, section 1).  Orders are odd 1..P_max in both branches plus c,
 * given as bit masks: bit b set <=> order 2b+1 present. */
typedef struct dpd_stream_desc {
    const void *in;          /* device complex64, n samples                  */
    void *out;               /* device complex64, n samples                  */
    int64_t n;               /* samples (>= 0)                               */
    uint32_t main_mask;      /* main-branch orders (bit b <=> order 2b+1)    */
    uint32_t conj_mask;      /* conjugate-branch orders                      */
    int32_t L;               /* taps, 1..16                                  */
    int32_t pad_;            /* zero                                         */
    const void *coeffs_dev;  /* device, K complex64 in section 2.2 layout    */
} dpd_stream_desc;

/* dpd_batch_create -- validate the descriptors, cut every stream into chunks
 * of 64*S samples (S = tune->samples_per_thread; a stream's last chunk may be
 * shorter), list them most expensive class first, upload the list (32 bytes
 * per chunk), and size the persistent grid.
 * `tune` may be NULL for the default launch shape.  The descriptor pointers
 * must stay valid for the life of the batch.  Synchronous on the host (the
 * chunk list and zeroed tables are in device memory on return; no device-wide
 * wait). */
dpd_status dpd_batch_create(const dpd_stream_desc *desc, int32_t n_streams, const dpd_tune *tune,
                            dpd_batch **out);

/* dpd_batch_apply -- one persistent launch (plus one coefficient-precombine
 * launch) on `stream`.  Allocates nothing, never synchronizes the host and
 * may be captured in a hipGraph (there is no device counter to reset).  Calls that overlap in time on one batch race. */
dpd_status dpd_batch_apply(dpd_batch *batch, void *stream);

/* dpd_batch_apply_each -- reference schedule: one launch per stream with the
 * same kernels as dpd_apply (for comparison against the persistent form). */
dpd_status dpd_batch_apply_each(dpd_batch *batch, void *stream);

/* dpd_batch_info -- number of chunks (full and ragged) in the persistent
 * launch and its number of blocks. */
dpd_status dpd_batch_info(const dpd_batch *batch, int64_t *n_tiles, int32_t *n_blocks);

/* dpd_batch_destroy -- frees the batch; freeing device memory waits for the
 * device, so kernels still reading the batch finish first. */
dpd_status dpd_batch_destroy(dpd_batch *batch);

/* --------------------------------------------------------------- training --
 * Helpers that let a coefficient-learning step (predistorter -> fixed PA
 * model -> loss -> backward -> Adam) run entirely in libdpd kernels.  Not in
 * the paper, whose training is offline least squares (section 2.2).
 *
 * dpd_loss_grad -- E = (1/n) sum_t |scale*y_t - x_t|^2 over n complex64
 * samples (y: PA output, x: the original input, scale: 1/PA gain), written as
 * one float to *loss_dev (device; may be NULL), and dE/dRe y + j dE/dIm y =
 * (2 scale / n)(scale*y - x) written to grad_y (device, n complex64; may be
 * NULL).  Deterministic (each thread sums in FP32 over at most 32 steps, then
 * in FP64; fixed-order FP64 sum of per-block partials).  ws: device workspace
 * of dpd_loss_ws_size() bytes, owned by the caller. */
dpd_status dpd_loss_ws_size(int64_t n, size_t *bytes);
dpd_status dpd_loss_grad(void *stream, const void *y, const void *x, int64_t n, float scale,
                         float *loss_dev, void *grad_y, void *ws, size_t ws_bytes);

/* dpd_adam_step -- one Adam update (Kingma & Ba) of `count` real parameters
 * in device memory (a complex coefficient vector is 2K interleaved floats):
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   p -= (lr / (1 - b1^step)) m / (sqrt(v / (1 - b2^step)) + eps).
 * step counts from 1.  m and v are caller-owned state (zero before step 1). */
dpd_status dpd_adam_step(void *stream, float *params, const float *grads, float *m, float *v,
                         int64_t count, int32_t step, float lr, float beta1, float beta2, float eps);

/* dpd_cascade_loss_grad -- the transmitter model of the learning loop as two
 * APH stages (Eq. 1 each) fused with the loss: per row, u = A(z) with A a
 * memoryless plan (L == 1: I/Q imbalance, LO leakage, static nonlinearity)
 * and y = B(u) with B a plan with memory (a PA), u taken as zero before the
 * row start; then E = (1/(rows n)) sum |scale*y - x|^2 into *loss_dev and
 * dE/dy = (2 scale / (rows n)) (scale*y - x) into grad_y, as dpd_loss_grad
 * computes from y.  u and y are never stored.  z, x, grad_y: device
 * complex64, rows x n at stride ld samples (ld >= n; ignored when rows == 1),
 * 8-byte aligned; grad_y must not overlap z or x.  ws: >= dpd_loss_ws_size
 * bytes.  DPD_EINVAL if A has more than one tap; DPD_EUNSUPPORTED if B has
 * orders above 7 or more than 4 taps (run the stages with dpd_apply_rows and
 * dpd_loss_grad instead).  Deterministic; allocates nothing.
 *
 * dpd_cascade_backward -- dE/dz from dE/dy through the same cascade: the
 * adjoint of B at u = A(z) (recomputed), then the adjoint of A, in the
 * complex-gradient convention of dpd_backward.  grad_z must not overlap z or
 * grad_y.  Same layout and limits. */
dpd_status dpd_cascade_loss_grad(const dpd_plan *A, const dpd_plan *B, void *stream, const void *z,
                                 const void *x, int64_t rows, int64_t n, int64_t ld, float scale,
                                 float *loss_dev, void *grad_y, void *ws, size_t ws_bytes);
dpd_status dpd_cascade_backward(const dpd_plan *A, const dpd_plan *B, void *stream, const void *z,
                                const void *grad_y, void *grad_z, int64_t rows, int64_t n, int64_t ld);

/* dpd_transmit_loss_grad -- the forward pass of the learning step in one
 * kernel: z = D(x) (Eq. 1 with predistorter plan P and, when coeffs_dev is not
 * NULL, the K complex64 device coefficients coeffs_dev, which the kernel
 * precombines itself with the arithmetic of dpd_apply_coeffs' table; the
 * plan's tables are not written), then u = A(z), y = B(u) and the loss
 * E and dE/dy of dpd_cascade_loss_grad (rows of x, z, grad_y at stride ld).
 * z is written for the cascade's adjoint (dpd_cascade_backward); z and grad_y
 * are bitwise those of dpd_apply_coeffs followed by dpd_cascade_loss_grad,
 * and E differs from it only in the order of the FP32 partial sums.  Built
 * for A memoryless with order 1 in each branch (I/Q imbalance and LO leakage)
 * and B with orders {1, 3, 5} and 3 taps (the PA of the learning workload),
 * and for P with orders up to 9 and up to 8 taps: other stages are
 * DPD_EUNSUPPORTED (run dpd_apply_coeffs and dpd_cascade_loss_grad).  x, z,
 * grad_y: device complex64, 8-byte aligned, z and grad_y not overlapping x or
 * each other.  ws: >= dpd_loss_ws_size bytes.  Allocates nothing. */
dpd_status dpd_transmit_loss_grad(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                  const void *coeffs_dev, const void *x, void *z, int64_t rows, int64_t n,
                                  int64_t ld, float scale, float *loss_dev, void *grad_y, void *ws,
                                  size_t ws_bytes);

/* dpd_transmit_backward -- the backward pass of the learning step: dE/dz
 * through the adjoint of the cascade (B at u = A(z), then A, as
 * dpd_cascade_backward computes it) and from it the predistorter's coefficient
 * gradient, dE/dcoeffs of Eq. (1) for the inputs x (as dpd_backward with
 * grad_x NULL computes it; the coefficients of P are not read).  In one
 * kernel when A is memoryless with order 1 in each branch, B has orders
 * {1, 3, 5} and 3 taps, P orders up to 9 and up to 8 taps, n is a multiple of
 * 256 and x, z, grad_y (and grad_z) are 16-byte aligned with an even row
 * stride: dE/dz then stays on chip.  Otherwise the two passes run with dE/dz
 * in grad_z, which must then be given (DPD_EUNSUPPORTED if it is NULL).
 *   x, z, grad_y  device complex64, rows x n at stride ld: the predistorter's
 *                 input and output and dE/dy (dpd_transmit_loss_grad writes z
 *                 and grad_y)
 *   grad_z        device, same layout, receives dE/dz, or NULL; must not
 *                 overlap x, z or grad_y
 *   grad_coeffs   device, receives the K complex64 gradients (required)
 *   ws, ws_bytes  device workspace of at least dpd_backward_ws_size(P) bytes
 * Deterministic (fixed-order reductions, FP64 finalisation).  Allocates
 * nothing. */
dpd_status dpd_transmit_backward(const dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream,
                                 const void *x, const void *z, const void *grad_y, void *grad_z,
                                 void *grad_coeffs, int64_t rows, int64_t n, int64_t ld, void *ws,
                                 size_t ws_bytes);

/* dpd_learn_step -- one whole coefficient-learning step in one call (three
 * launches): the one-pass forward of dpd_transmit_loss_grad with the
 * coefficients coeffs_dev, the one-pass backward of dpd_transmit_backward,
 * then one launch that finalises the loss and the gradient (FP64, as those
 * calls do) and applies the Adam update of dpd_adam_step to coeffs_dev in
 * place.  Results are bitwise those of the three calls followed by
 * dpd_adam_step.  Arguments as there:
 *   coeffs_dev       K complex64 (device), read, then updated
 *   adam_m, adam_v   2K floats each (device), Adam moments (zero before
 *                    step 1), updated; step counts from 1
 *   x, z, grad_y     rows x n at stride ld (device complex64): the input and
 *                    the buffers for z and dE/dy
 *   loss_dev         receives E (the loss at the coefficients before the
 *                    update), or NULL
 *   grad_coeffs      receives dE/dcoeffs (K complex64), or NULL
 *   ws, ws_bytes     at least dpd_learn_step_ws_size(P) bytes
 * Built for the shapes of the one-pass kernels (stages as in
 * dpd_transmit_loss_grad; n a multiple of 256; x, z, grad_y 16-byte aligned
 * with an even row stride): others are DPD_EUNSUPPORTED (use the separate
 * calls).  coeffs_dev, adam_m, adam_v and grad_coeffs must not overlap.
 * Allocates nothing; no host synchronization. */
dpd_status dpd_learn_step_ws_size(const dpd_plan *P, size_t *bytes);
dpd_status dpd_learn_step(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream, void *coeffs_dev,
                          float *adam_m, float *adam_v, int32_t step, float lr, float beta1, float beta2,
                          float eps, const void *x, void *z, void *grad_y, int64_t rows, int64_t n, int64_t ld,
                          float scale, float *loss_dev, void *grad_coeffs, void *ws, size_t ws_bytes);

/* dpd_learn_step_dev -- dpd_learn_step with Adam's step count in device
 * memory, for learning loops captured into a graph: *step_dev (one int32,
 * 4-byte aligned, 0 before the first step) is advanced by one on the device,
 * in stream order, before the update uses it, so every replay of a captured
 * call takes the next step.  The bias corrections 1 - beta^t are computed on
 * the device in FP64 (dpd_learn_step computes them on the host: results can
 * differ from it in the last bit).  step_dev must not overlap the other
 * buffers; NULL is DPD_EINVAL.  Otherwise as dpd_learn_step. */
dpd_status dpd_learn_step_dev(dpd_plan *P, const dpd_plan *A, const dpd_plan *B, void *stream, void *coeffs_dev,
                              float *adam_m, float *adam_v, int32_t *step_dev, float lr, float beta1, float beta2,
                              float eps, const void *x, void *z, void *grad_y, int64_t rows, int64_t n, int64_t ld,
                              float scale, float *loss_dev, void *grad_coeffs, void *ws, size_t ws_bytes);

/* ------------------------------------------------------- least squares --
 * The paper's coefficient estimate (section 2.2, Eq. 2): with the plan's
 * basis, row m of Psi is
 *   [psi_p(y_{m-k}) for main orders p, taps k; conj(psi_q(y_{m-k})) for
 *    conjugate orders q, taps k; 1]
 * in the coefficient stacking of section 2.2 (K columns), samples before each
 * row start taken as zero (the first n rows of the zero-filled element
 * matrices of Eq. 2, per row).  The least-squares coefficients solve
 *   (Psi^H Psi) h = Psi^H t.
 * In the indirect-learning use, y is the PA output divided by its gain and t
 * the PA input (the predistorter output); the fitted postdistorter is then
 * copied into the predistorter.
 *
 * dpd_ls_ws_size -- workspace bytes for dpd_ls_normal on rows x n samples.
 *   DPD_EUNSUPPORTED if 2K+2 > 192 (K > 95): the Gram kernel holds at most
 *   12 x 12 tiles of 16 x 16.
 *
 * dpd_ls_normal -- A = Psi^H Psi (K x K complex128, row-major, Hermitian) and
 *   b = Psi^H t (K complex128), summed over all rows, with Psi built from
 *   y_scale * y (e.g. 1 / PA gain; finite).  y, t: device complex64,
 *   rows x n at stride ld samples (ld >= n; ignored when rows == 1), 8-byte
 *   aligned.  ws: device, >= dpd_ls_ws_size bytes, 256-byte aligned,
 *   caller-owned scratch.  A, b: device, 8-byte aligned, overwritten.  FP32
 *   features, each split into a bf16 high and low part for the matrix cores
 *   (all four cross products summed in FP32: FP32-level accuracy),
 *   accumulated in FP32 over slabs of 1024 to 8192 samples (the size
 *   depends only on rows, n and the device's CU count), the slabs summed in
 *   FP64 in a fixed order: deterministic.  Allocates nothing, does not
 *   synchronize; rows * n == 0 gives A = 0, b = 0.  The first call on a plan
 *   also picks the order of the basis entries in the kernel's shared-memory
 *   rows (host work, once per plan, a few milliseconds at most; safe when
 *   several threads make the first call together). */
dpd_status dpd_ls_ws_size(const dpd_plan *plan, int64_t rows, int64_t n, size_t *bytes);
dpd_status dpd_ls_normal(dpd_plan *plan, void *stream, const void *y, const void *t, int64_t rows,
                         int64_t n, int64_t ld, float y_scale, void *ws, size_t ws_bytes, void *A, void *b);

/* dpd_ls_solve -- solve (A + delta I) h = b by Cholesky in FP64 on the device,
 *   delta = ridge * mean(Re diag A) (ridge >= 0; 0 for the plain normal
 *   equations).  A: K x K complex128 Hermitian (only the lower triangle is
 *   read), b: K complex128, both device, 16-byte aligned.  h: device, K
 *   complex64 (the section 2.2 stacking, ready for dpd_set_coeffs_device).
 *   info: device int32, set to 0 on success or j+1 when the pivot of column j
 *   is not positive (h is then NaN); the host sees it after synchronizing.
 *   ws: device, >= dpd_ls_solve_ws_size bytes (K*K complex128), 16-byte
 *   aligned (used for K > 64; smaller systems are factored in shared
 *   memory).  One workgroup (four wavefronts up to K = 56, one beyond);
 *   DPD_EUNSUPPORTED for K > 1024. */
dpd_status dpd_ls_solve_ws_size(int32_t K, size_t *bytes);
dpd_status dpd_ls_solve(void *stream, int32_t K, const void *A, const void *b, double ridge, void *ws,
                        size_t ws_bytes, void *h, void *info);

/* ------------------------------------------------------------ measurement --
 * dpd_copy -- out[t] = in[t] for t = 0..n-1 (complex64, device, 16-byte
 * aligned, not overlapping) with the memory walk of the forward kernel and
 * none of its arithmetic: the practical HBM ceiling of that walk, which the
 * benchmark reports beside the filter's rate (not part of the paper's
 * method).  Asynchronous on `stream`; allocates nothing. */
dpd_status dpd_copy(void *stream, const void *in, void *out, int64_t n);

/* ------------------------------------------------------------------- misc -- */
const char *dpd_status_string(dpd_status status);
int dpd_last_hip_error(void);
const char *dpd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DPD_H */
