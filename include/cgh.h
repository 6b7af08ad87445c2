/*
 * cgh.h -- C ABI of libcgh, MI355X (gfx950) progressive saliency-guided
 * hologram generation.
 *
 * Method: "Progressive hologram generation based on object saliency"
 * (arXiv 2211.09938).  An object is decomposed by a multi-level Haar DWT
 * (Sec. 2, Eq. 2, algorithm step 1); the coarsest approximation is rendered
 * for every block and the detail coefficients of level l only in blocks whose
 * block-maximum saliency exceeds that level's threshold (steps 2-5, Sec. 3
 * thresholds); every coefficient is scaled onto the fringe of its basis block
 * and superposed on the hologram plane (Eq. 3).  The fringe is the point-source
 * object wave of Eq. 1 in Fresnel form,
 *     kernel(dy, dx) = exp(i*pi*pitch^2*(dx^2 + dy^2) / (lambda*z)),
 * object and hologram sharing one pixel grid of pitch `pitch`.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers unless marked [host].  Images are
 *    row-major, index [y][x], y = row (ny rows, nx columns).
 *  - Complex arrays are interleaved (re, im) float pairs, i.e. the memory
 *    layout of C99 float complex / torch.complex64; `float* h` holds 2*ny*nx
 *    floats.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on `stream`; none synchronises it.
 *  - The caller owns every buffer.  The library never allocates, frees or
 *    retains caller memory; scratch memory comes from the caller's
 *    `workspace`, sized by cgh_workspace_size().
 *  - Every argument is validated on the host before anything is enqueued.
 *    On an error return nothing has been enqueued and no output is touched.
 *    A failed launch returns CGH_ERROR_HIP; cgh_last_hip_error() gives the
 *    hipError_t of the calling thread's last such failure.
 *  - Limits: 1 <= levels <= 3 (the paper uses three levels: 8x8, 4x4, 2x2
 *    and 1x1 block fringes); ny and nx divisible by 2^levels and at most
 *    CGH_MAX_SIDE; 1 <= n_layers <= 256.  ny == 0 or nx == 0 is an empty
 *    problem: success, nothing enqueued.
 */
#ifndef CGH_H
#define CGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGH_MAX_SIDE 16384
#define CGH_MAX_LAYERS 256
#define CGH_MAX_LEVELS 3

typedef enum {
    CGH_SUCCESS = 0,
    CGH_ERROR_INVALID_VALUE = 1, /* NULL required pointer, non-finite/non-positive optics, bad flag */
    CGH_ERROR_SHAPE = 2,         /* side not divisible by 2^levels, too large, levels out of range */
    CGH_ERROR_UNSUPPORTED = 3,   /* a valid request this build does not implement */
    CGH_ERROR_OUT_OF_MEMORY = 4, /* plan creation could not allocate */
    CGH_ERROR_WORKSPACE = 5,     /* workspace NULL or smaller than cgh_workspace_size() */
    CGH_ERROR_HIP = 6,           /* a HIP runtime call or launch failed */
    CGH_ERROR_INTERNAL = 7,      /* a launch would not fit the workspace layout the library
                                    computed itself: a library defect, reported before
                                    anything is enqueued */
    CGH_ERROR_SCRATCH_LIMIT = 8  /* cgh_progressive_hologram_noalloc: the problem needs more
                                    scratch than CGH_NOALLOC_SCRATCH_BYTES */
} cgh_status;

/* Arithmetic of the two dense contractions (the coefficient stage and the
 * fringe look-up tables are always built from FP64 phases). */
typedef enum {
    CGH_FP32 = 0,       /* FP32 operands, FP32 MFMA, FP32 accumulate            */
    CGH_BF16_SPLIT = 1, /* each operand v = hi + lo, hi = bf16(v), lo = bf16(v-hi);
                           products hi*hi + hi*lo + lo*hi on bf16 MFMA, FP32 acc  */
    CGH_FP16_SPLIT = 2  /* same with fp16 halves                                */
} cgh_precision;

enum {
    CGH_FLAG_ACCUMULATE = 1u,   /* hologram += result instead of hologram = result */
    CGH_FLAG_EQ1_PREFACTOR = 2u /* multiply layer d by exp(i*2*pi*z_d/lambda)/z_d,
                                   the constant of Eq. 1's paraxial expansion     */
};

/* Human-readable name of a status code (static storage, never NULL). */
const char* cgh_status_string(int status);

/* hipError_t of this thread's last CGH_ERROR_HIP return (0 if none). */
int cgh_last_hip_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int cgh_version(void);

/*
 * Multi-level 2D averaging Haar analysis (Sec. 2, Eq. 2; algorithm step 1).
 * Per axis lo = (a+b)/2, hi = (a-b)/2, x first then y, recursing on LL.
 * Output in Mallat layout: inside the top-left (2h x 2w) square of each level,
 * [0:h,0:w] LL, [0:h,w:2w] V (lo_y hi_x), [h:2h,0:w] H (hi_y lo_x),
 * [h:2h,w:2w] D (hi_y hi_x).  The level-`levels` LL is the 2^levels-block mean.
 * x: ny*nx floats (input), coeffs: ny*nx floats (output, must not alias x).
 * Bit-exact with the FP64 definition whenever the input values are dyadic.
 */
int cgh_haar_dwt(const float* x, int ny, int nx, int levels, float* coeffs, void* stream);

/* Inverse of cgh_haar_dwt: a = lo + hi, b = lo - hi, y first then x per level. */
int cgh_haar_idwt(const float* coeffs, int ny, int nx, int levels, float* x, void* stream);

/*
 * Bytes of device workspace that cgh_progressive_hologram,
 * cgh_hologram_backward and cgh_fresnel_backpropagate need for this problem.
 * bytes: [host] output.
 */
int cgh_workspace_size(int ny, int nx, int n_layers, int levels, int precision, size_t* bytes);

/* How a workspace of cgh_workspace_size() bytes is divided (diagnostics). */
typedef struct {
    size_t total;           /* cgh_workspace_size()                                        */
    size_t shared_bytes;    /* region shared by the paths' operand panels and scratch      */
    size_t partial_bytes;   /* split-K partial holograms                                   */
    int split_reserved;     /* partial holograms the layout holds room for                 */
    int split_second;       /* K split of this precision's single-scene second contraction */
    size_t forward_bytes;   /* forward operand panels (cgh_progressive_hologram, stages)   */
    size_t backward_bytes;  /* adjoint panels, partials and tables (cgh_hologram_backward) */
    size_t backprop_bytes;  /* back-propagation panels (cgh_fresnel_backpropagate)         */
    size_t literal_bytes;   /* cgh_literal_hologram panels                                 */
    size_t fused_bytes;     /* cgh_fused_hologram panels and reconstruction                */
    size_t lut_x_offset;    /* byte offset of the x fringe tables (float): per layer d, level
                               l, band b (0 lo, 1 hi), part (0 re, 1 im), table
                               ((d*levels + l-1)*2 + b)*2 + part of 2*nx floats, entry i
                               holding the fringe at offset i - nx (Sec. 2 LUT blocks)     */
    size_t lut_y_offset;    /* the y tables, 2*ny floats each, times the layer's prefactor */
    size_t gen_x_offset;    /* the x level tables in the operand format of the call's
                               precision, written by the forward pass: per (layer d, level l)
                               three bands of 2*nx entries of 8 bytes, starting at entry
                               (d*levels + l-1)*3*2*nx -- band 0 (lo), band 1 (hi), zeros;
                               an entry is (re, im) as FP32, or for the split forms the words
                               hi | lo << 16 of re and of im (hi = RNE16(v), lo =
                               RNE16(v - hi))                                              */
    size_t gen_y_offset;    /* the y tables in that format, 2*ny entries per band          */
    size_t koff_row_offset; /* per (layer, level), beside each active coefficient row i of
                               the forward pass its offset into the y operand-format tables
                               (i < ny/2^l: -i*2^l; else 2*ny - (i - ny/2^l)*2^l), ints, and
                               3*ny up to the next multiple of 16 rows; one segment per
                               (layer, level) of the level's side ny/2^(l-1) rounded up to 16,
                               layer-major                                                 */
    size_t koff_col_offset; /* the same for the active columns, over nx                    */
} cgh_layout_info;

/* Fills *info [host] for the problem; errors as cgh_workspace_size(). */
int cgh_workspace_layout(int ny, int nx, int n_layers, int levels, int precision,
                         cgh_layout_info* info);

/*
 * Progressive saliency-guided hologram (Sec. 2, Eqs. 1-3, steps 1-5):
 *   A_d    = object * [layer_index == d]                     (3D extension, Sec. 2)
 *   C_d    = W(A_d) with level-l details zeroed where maxpool_{2^l}(saliency) <= t_l
 *   H      = sum_d P_d * sum_coefficients C_d * (fringe of the coefficient's basis block)
 * which equals the Fresnel sum of the masked reconstruction S(C_d) of every layer.
 *
 *  object       ny*nx float amplitudes.
 *  layer_index  ny*nx uint8 in [0, n_layers), or NULL: every pixel in layer 0
 *               (then n_layers must be 1).  Values >= n_layers belong to no layer.
 *  z            [host] n_layers distances in metres, finite and > 0.
 *  saliency     ny*nx floats, or NULL: every block salient.
 *  thresholds   [host] `levels` floats in [0,1], t_1 (finest details) first, or
 *               NULL: (0.9, 0.7, 0.5) for 3 levels (Sec. 3), 0.5 per level otherwise.
 *               A level-l detail is kept iff its block maximum is strictly greater.
 *  lambda, pitch  metres, finite and > 0.
 *  precision    cgh_precision.   flags: CGH_FLAG_*.
 *  workspace    device scratch of at least cgh_workspace_size() bytes.
 *  hologram     2*ny*nx floats (complex64 interleaved), overwritten (or
 *               accumulated into with CGH_FLAG_ACCUMULATE).  Must not alias inputs.
 */
int cgh_progressive_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                             const double* z, const float* saliency, const float* thresholds,
                             double lambda, double pitch, int ny, int nx, int levels,
                             int precision, unsigned flags, void* workspace,
                             size_t workspace_bytes, float* hologram, void* stream);

/*
 * Allocation-free variant of cgh_progressive_hologram, for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same method, kernels
 * and results as cgh_progressive_hologram (bit-identical for the same
 * arguments); the scratch comes from a library-resident device array of
 * CGH_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends.  The call allocates and frees nothing.
 *  - Problems whose forward-pass scratch exceeds CGH_NOALLOC_SCRATCH_BYTES are
 *    rejected with CGH_ERROR_SCRATCH_LIMIT before anything is enqueued
 *    (128 MiB holds a 1024 x 1024 single-layer problem, or 512 x 512 with two
 *    layers; 2048 x 2048 does not fit).
 *  - Every call on one GPU uses that GPU's single array: calls that overlap on
 *    one GPU (other streams, other threads, a graph replayed while another
 *    call runs) race and give undefined results.  Serialise them.  Each call
 *    clears what it needs cleared; nothing carries over between calls.
 *  - The array's device address is looked up on a device's first call (with
 *    that device current); a failure there returns CGH_ERROR_HIP.
 * Arguments, other errors and ownership as for cgh_progressive_hologram,
 * without the workspace; profiling (cgh_profile_enable) does not apply.
 */
#define CGH_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int cgh_progressive_hologram_noalloc(const float* object, const uint8_t* layer_index,
                                     int n_layers, const double* z, const float* saliency,
                                     const float* thresholds, double lambda, double pitch,
                                     int ny, int nx, int levels, int precision, unsigned flags,
                                     float* hologram, void* stream);

/*
 * Progressive stage holograms (Sec. 2, steps 2-5; the progressive display of
 * Sec. 3): levels+1 cumulative holograms written one after the other,
 *   stages[0]      the level-L approximation alone (every block, step 2),
 *   stages[j]      stages[j-1] + the salient details of level L-j+1 (steps 3-5),
 *   stages[levels] the full progressive hologram of cgh_progressive_hologram
 *                  (equal up to FP32 summation order).
 * stages: (levels+1)*2*ny*nx floats, complex64 interleaved, overwritten; must
 * not alias the inputs.  The workspace is the one cgh_workspace_size() gives
 * for the same arguments; the stages run one after the other in stream order
 * and reuse it.  CGH_FLAG_ACCUMULATE is rejected; other arguments, errors and
 * ownership as for cgh_progressive_hologram.
 */
int cgh_progressive_stages(const float* object, const uint8_t* layer_index, int n_layers,
                           const double* z, const float* saliency, const float* thresholds,
                           double lambda, double pitch, int ny, int nx, int levels, int precision,
                           unsigned flags, void* workspace, size_t workspace_bytes, float* stages,
                           void* stream);

/*
 * Paper-literal form of the progressive hologram (Sec. 2, steps 2-5 in the
 * image domain): the coarsest approximation image (2^L x 2^L block means) and
 * the residual map of every level (finer approximation image minus the coarser
 * one replicated 2 x 2, kept where the level's quantised saliency is above its
 * threshold), each point multiplied onto the Fresnel fringe of a uniform block
 * of its size and added at its position.  The result equals
 * cgh_progressive_hologram up to rounding order (a cross-check of the
 * coefficient form); the work is dense, one contraction per image and level
 * with inner dimension N/2^L, ..., N/2, N (no saliency skipping).  Arguments,
 * flags, workspace (cgh_workspace_size), errors and ownership as for
 * cgh_progressive_hologram.
 */
int cgh_literal_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                         const double* z, const float* saliency, const float* thresholds,
                         double lambda, double pitch, int ny, int nx, int levels, int precision,
                         unsigned flags, void* workspace, size_t workspace_bytes, float* hologram,
                         void* stream);

/*
 * Dense form of the same hologram (the "reconstruct, then contract" ablation):
 * by linearity (Eq. 3) the sum over coefficients of coefficient x block
 * fringe is the Fresnel hologram of each layer's masked reconstruction
 * A_d = S(M W(object * [layer == d])) (Sec. 2 steps 2-5 summed), so this
 * computes A_d with the inverse Haar transform and then
 *   H (+)= sum_d P_d * K_y A_d K_x^T,   K[m][q] = exp(i pi p^2 (m - q)^2 / (lambda z_d)),
 * two dense products per layer with inner dimensions nx and ny: 12 N^3 real
 * flops per layer for N x N, against 18 N^3 for the per-level dense form and
 * the saliency-compacted work of cgh_progressive_hologram.  Equals
 * cgh_progressive_hologram up to rounding order.  Arguments, flags,
 * workspace (cgh_workspace_size), errors and ownership as for
 * cgh_progressive_hologram.
 */
int cgh_fused_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                       const double* z, const float* saliency, const float* thresholds,
                       double lambda, double pitch, int ny, int nx, int levels, int precision,
                       unsigned flags, void* workspace, size_t workspace_bytes, float* hologram,
                       void* stream);

/*
 * Eq. 1 with the exact distance (no Fresnel approximation), for measuring
 * the error of the Fresnel form of the hot path:
 *   hologram[y][x] = sum_d sum_{q,p} Ahat_d[q][p] / r * exp(i 2 pi r / lambda),
 *   r = sqrt(pitch^2 ((x-p)^2 + (y-q)^2) + z_d^2),
 * with Ahat_d the same masked reconstruction of layer d as in
 * cgh_progressive_hologram (whose result with CGH_FLAG_EQ1_PREFACTOR is the
 * Fresnel approximation of this sum).  Direct sum: ny*nx*ny*nx*n_layers
 * terms (at most; zero points are skipped), FP64 reduction of the large phase
 * term, FP32 elsewhere, FP64 summation of 64-point partial sums.
 * flags: CGH_FLAG_ACCUMULATE only (CGH_FLAG_EQ1_PREFACTOR is rejected: the
 * exact sum already carries the phase and 1/r of Eq. 1).  Workspace as
 * cgh_workspace_size(ny, nx, n_layers, levels, any precision).  Other
 * arguments, errors and ownership as for cgh_progressive_hologram.
 */
int cgh_exact_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                       const double* z, const float* saliency, const float* thresholds,
                       double lambda, double pitch, int ny, int nx, int levels, unsigned flags,
                       void* workspace, size_t workspace_bytes, float* hologram, void* stream);

/*
 * Adjoint of cgh_progressive_hologram with respect to the object amplitudes.
 * grad_hologram: 2*ny*nx floats, G = dL/dRe(H) + i dL/dIm(H) (the cotangent
 * torch hands to a complex output).  Writes grad_object (ny*nx floats):
 *   dL/dA[q,p] = [ S M W ( Re( P_d * sum_{y,x} conj(G[y,x]) kernel_d(y-q, x-p) ) ) ][q,p],
 *   d = layer_index[q,p]   (zero for pixels in no layer),
 * using that the masked averaging-Haar reconstruction S M W is self-adjoint.
 * Other arguments as for cgh_progressive_hologram (CGH_FLAG_ACCUMULATE is
 * rejected).
 */
int cgh_hologram_backward(const float* grad_hologram, const uint8_t* layer_index, int n_layers,
                          const double* z, const float* saliency, const float* thresholds,
                          double lambda, double pitch, int ny, int nx, int levels, int precision,
                          unsigned flags, void* workspace, size_t workspace_bytes,
                          float* grad_object, void* stream);

/*
 * Fresnel back-propagation of a hologram to the object plane at distance z
 * (numerical reconstruction, Sec. 2 last paragraph, here with the same Fresnel
 * kernel as the forward pass):
 *   adjoint == 0:  out[q,p] = 1/(ny*nx) * sum_{y,x} conj(kernel(y-q, x-p)) * in[y,x]
 *   adjoint != 0:  out[y,x] = 1/(ny*nx) * sum_{q,p} kernel(y-q, x-p) * in[q,p]
 * field_in, field_out: 2*ny*nx floats complex, must not alias.  The workspace
 * is sized by cgh_workspace_size(ny, nx, 1, 1, precision, ...).
 */
int cgh_fresnel_backpropagate(const float* field_in, int ny, int nx, double lambda, double pitch,
                              double z, int precision, int adjoint, void* workspace,
                              size_t workspace_bytes, float* field_out, void* stream);

/*
 * Angular-spectrum propagation of a complex field over distance z (metres,
 * any sign).  The paper reconstructs its holograms with the inverse
 * angular-spectrum method at the scene parameters (Sec. 2, end of the method):
 * that is this operator with z -> -z, the hologram as `field` and the object
 * plane in `out`.
 *   out = IDFT2( DFT2(field) * T ),
 *   T(fx, fy) = exp(i 2 pi z sqrt(1/lambda^2 - fx^2 - fy^2)), 0 where the root is
 *   imaginary (evanescent),  fx = kx / (nx pitch), kx in [-nx/2, nx/2) in DFT order,
 * DFT2 unnormalised, IDFT2 scaled by 1/(ny nx); the grid is the field's own (no
 * padding: the DFT's periodic wrap-around is part of the operator).
 *  field, out   [device] 2*ny*nx floats, complex64 interleaved, row-major; may be
 *               the same array (in place).
 *  ny, nx       2^a or 3*2^a in [2, 4096] (CGH_ERROR_SHAPE otherwise; 0: no-op).
 *  lambda, pitch  finite, > 0; z finite.
 *  workspace    [device] at least cgh_angular_spectrum_workspace_size(ny, nx) bytes.
 * FP32 FFTs with FP64 twiddle tables and an FP64 transfer phase.
 */
size_t cgh_angular_spectrum_workspace_size(int ny, int nx);  /* 0 for unsupported sides */
int cgh_angular_spectrum(const float* field, int ny, int nx, double lambda, double pitch, double z,
                         void* workspace, size_t workspace_bytes, float* out, void* stream);

/* Work counts of a forward pass: of the last cgh_progressive_hologram that used
 * a workspace (cgh_workspace_stats), or summed over a plan's scenes
 * (cgh_plan_get_stats). */
typedef struct cgh_stats_s {
    long long k_active;          /* active K of the second contraction: for every layer and
                                    level, the nonzero rows of its coefficient square, or its
                                    nonzero columns where the level is contracted columns-first
                                    (Eq. 3 in the other order; taken where the padded column
                                    count is the smaller)                                      */
    long long k_padded;          /* K the second contraction ran over (segments padded to 16)  */
    long long k_total;           /* K of the dense form (every row of every level and layer)   */
    int k_tile;                  /* K tile of the contractions                                 */
    int split_k;                 /* K-range split of the second contraction                    */
    double flops_first;          /* algorithmic real flops, first contraction: 4 x the sum over
                                    (layer, level) of active rows x active columns x nx
                                    (rows-first) or x ny (columns-first)                       */
    double flops_second;         /* algorithmic real flops, second contraction:
                                    8 * ny * nx * k_active                                     */
    double flops_second_issued;  /* 8 * ny * nx * k_padded: the count on the padded K (FP32
                                    runs three real products per complex product there, i.e.
                                    3/4 of it on the matrix cores)                          */
    long long operators[4];      /* operator count of Sec. 3 per progressive step, for one image
                                    plane (the saliency masks are shared by the layers):
                                    [0] the approximation, one per point of the (ny/2^L) x
                                    (nx/2^L) image; [j] the residual-map points of level L-j+1
                                    whose block is salient (4 per salient detail position);
                                    entries beyond `levels` are 0                             */
    long long operators_pointwise; /* ny * nx: one operator per object point                   */
} cgh_stats;

/* ---------------------------------------------------------- batched plans */

/*
 * One scene of a batch: the arguments of cgh_progressive_hologram that vary per
 * scene.  Device pointers as there; z is [host] and is copied at plan creation.
 * The device buffers must stay valid (and unmoved) for the plan's lifetime:
 * the plan's captured graph reads and writes them on every execution.
 */
typedef struct {
    const float* object;         /* ny*nx */
    const uint8_t* layer_index;  /* ny*nx, or NULL (then n_layers == 1) */
    int n_layers;
    const double* z;             /* [host] n_layers distances in metres */
    const float* saliency;       /* ny*nx, or NULL */
    int ny, nx;
    float* hologram;             /* 2*ny*nx floats (complex64), overwritten */
} cgh_scene;

typedef struct cgh_plan cgh_plan;

/*
 * Plans many scenes of uneven size as one unit (the batched form of
 * cgh_progressive_hologram; same method, same arguments per scene).  The plan
 * owns device memory for every scene's workspace, merges the contraction
 * problems of all scenes into one table per contraction, runs each contraction
 * as one persistent launch whose workgroups pull tiles from a shared counter,
 * and captures the whole batch into a HIP graph.  Tile shapes come from an
 * autotuner that times the candidates on this batch (for the split forms'
 * second contraction also the one-workgroup-per-CU 256 x 128 kernel, launched
 * over every scene's tiles) and caches the winners, as
 * JSON lines keyed by GPU architecture, precision and batch signature, in
 * tune_cache_path (NULL: no cache; the file is created if missing).
 * Plan creation synchronises `stream` (it runs the batch while tuning).
 * Errors: as cgh_progressive_hologram per scene, CGH_ERROR_OUT_OF_MEMORY if
 * the device memory cannot be allocated.  *plan is NULL on error.
 */
int cgh_plan_create(const cgh_scene* scenes /* [host] */, int n_scenes, int levels, double lambda,
                    double pitch, const float* thresholds, int precision, unsigned flags,
                    const char* tune_cache_path, void* stream, cgh_plan** plan /* [host] */);

/* Launches the captured graph on `stream`: every scene's hologram is
 * recomputed from the current contents of its input buffers.  While stage
 * profiling is on (cgh_profile_enable) the same kernels are launched eagerly
 * instead, with event pairs around the per-scene stages (CGH_STAGE_PLAN) and
 * the two persistent contractions (CGH_STAGE_FIRST, CGH_STAGE_SECOND). */
int cgh_plan_execute(cgh_plan* plan, void* stream);

/* Frees the plan (waits for nothing: the caller synchronises first). */
int cgh_plan_destroy(cgh_plan* plan);

typedef struct {
    int n_scenes;
    int first_tile[2];     /* rows, cols of the first contraction's tile  */
    int second_tile[2];    /* rows, cols of the second contraction's tile */
    int from_cache;        /* tile shapes read from the tune cache         */
    int persistent_grid;   /* workgroups of each persistent launch         */
    double tune_ms_first;  /* measured time of the chosen first contraction (ms, 0 if cached) */
    double tune_ms_second;
    size_t device_bytes;   /* device memory the plan owns                  */
} cgh_plan_info;

int cgh_plan_get_info(const cgh_plan* plan, cgh_plan_info* info /* [host] */);

/* Work counts of the plan's last execution, summed over its scenes (the
 * cgh_stats of every scene added up; split_k = 1).  Synchronises `stream`. */
int cgh_plan_get_stats(const cgh_plan* plan, cgh_stats* stats /* [host] */, void* stream);

/* ------------------------------------------------------------ diagnostics */

/* Stages of cgh_progressive_hologram, in launch order. */
enum {
    CGH_STAGE_COEF = 0,    /* flag clear + fused layer split / Haar / saliency / masking   */
    CGH_STAGE_LUT = 1,     /* FP64 fringe tables, both axes                                 */
    CGH_STAGE_PLAN = 2,    /* active row/column lists, plan, K-contiguous operand panels    */
    CGH_STAGE_FIRST = 3,   /* first contraction  T_{d,l} = Cb_{d,l} Fx_{d,l}^T (active rows) */
    CGH_STAGE_SECOND = 4,  /* second contraction H = sum_{d,l} Fy_{d,l} T_{d,l}             */
    CGH_STAGE_REDUCE = 5,  /* split-K partial sum (only when the K range is split)          */
    CGH_STAGE_COUNT = 6
};

/* Per-stage timing of cgh_progressive_hologram: on != 0 makes every later
 * call record a HIP event pair around each stage, on the call's own stream
 * (events come from a library-owned pool).  Process-wide, thread-safe. */
int cgh_profile_enable(int on);

/* Restricts the stages that record event pairs while profiling is on to those
 * whose bit (1u << CGH_STAGE_*) is set in mask; the default is every stage.
 * Each recorded event idles the stream for a few microseconds, so a timed loop
 * that needs one stage's duration brackets only that stage.  Process-wide,
 * thread-safe; never fails. */
int cgh_profile_stages(unsigned mask);

/* Waits for every recorded event pair, adds the elapsed times to per-stage
 * totals and returns them: ms[CGH_STAGE_COUNT] milliseconds and
 * launches[CGH_STAGE_COUNT] event pairs, both [host], either may be NULL.
 * reset != 0 clears the totals after reading. */
int cgh_profile_read(double* ms, long long* launches, int reset);


/* Reads the plan back from `workspace` (same problem arguments as the forward
 * call) and fills *stats [host].  Synchronises `stream`. */
int cgh_workspace_stats(const void* workspace, int ny, int nx, int n_layers, int levels,
                        int precision, cgh_stats* stats, void* stream);

/* Instruction of the matrix-core throughput probe. */
enum {
    CGH_PEAK_FP32 = 0, /* v_mfma_f32_32x32x2f32:     4096 flops per instruction  */
    CGH_PEAK_BF16 = 1, /* v_mfma_f32_32x32x16_bf16: 32768 flops per instruction */
    CGH_PEAK_FP16 = 2  /* v_mfma_f32_32x32x16_f16:  32768 flops per instruction */
};

/*
 * Matrix-core throughput probe (diagnostics; not part of the method): what the
 * matrix cores of this GPU sustain under dense load, the attainable rate beside
 * the published peak.  Launches `blocks` workgroups of four waves; each wave
 * runs iters x 32 MFMAs of `kind` on eight independent register accumulators
 * (no memory access inside the loop), then every thread writes one float of
 * its accumulator sum to sink.
 *  zero_operands  0: pseudo-random operands of magnitude [0.5, 2), four A and
 *                 four B sets in rotation, so the operand bits change from one
 *                 MFMA to the next as in a contraction; 1: all-zero operands.
 *  blocks         1 .. 1048576 (256 = one wave per SIMD on 256 CUs).
 *  iters          1 .. 16777216.
 *  sink           [device] blocks*256 floats, overwritten.
 *  flops          [host] out: real flops of the launch, 2*M*N*K per MFMA.
 * Errors: CGH_ERROR_INVALID_VALUE for an unknown kind, counts out of range or a
 * NULL pointer (nothing launched); CGH_ERROR_HIP for a failed launch.
 */
int cgh_mfma_peak(int kind, int zero_operands, int blocks, int iters, float* sink, double* flops,
                  void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CGH_H */
