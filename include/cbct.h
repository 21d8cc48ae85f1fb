/*
 * cbct.h -- C ABI of the MI355X (gfx950) hot path of PICCS-regularised Krylov
 * cone-beam CT reconstruction (Hastings, Islam, Sabate Landman, Hatamikia,
 * Schoenlieb, Biguri: "Real-time CBCT reconstructions using Krylov solvers in
 * repeated scanning procedures").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns an int status (CBCT_OK or a negative CBCT_ERR_*); nothing
 *   throws or aborts across the ABI.  cbct_last_error() returns a thread-local
 *   message for the last failure on the calling thread.
 * - Device calls take a hipStream_t passed as void* (NULL = the null stream).
 *   They validate their arguments synchronously, enqueue their kernels on that
 *   stream and return; results are ready when the stream reaches that point.
 *   A device fault surfaces as CBCT_ERR_DEVICE at a later call or when the
 *   caller synchronises the stream.
 * - Pointers named x, y, b, xp, w1, w2, workspace are DEVICE pointers owned by
 *   the caller; the library never frees caller memory and keeps no reference
 *   to it after the call's kernels have run.
 * - Layouts: volumes are x[z][y][x] (x fastest), nx*ny*nz float32;
 *   projections are y[view][v][u] (u fastest), n_views*nv*nu float32.
 *
 * Geometry (reading of the paper's unstated conventions): world frame in mm,
 * origin at the isocentre, z = rotation axis.  Voxel (i,j,k) is the box
 * [-n_a h_a/2 + i h_a, -n_a h_a/2 + (i+1) h_a] per axis.  View angle th: source
 * S = (DSO cos th, DSO sin th, 0), flat detector centred at
 * ((DSO-DSD) cos th, (DSO-DSD) sin th, 0) with axes e_u = (-sin th, cos th, 0)
 * and e_v = (0, 0, 1); pixel (iu, iv) is centred at
 * ((iu+1/2) du - nu du/2) e_u + ((iv+1/2) dv - nv dv/2) e_v from there.
 */
#ifndef CBCT_H
#define CBCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBCT_OK 0
#define CBCT_PENDING 1        /* server poll: request not finished yet        */
#define CBCT_ERR_INVALID -1   /* bad argument, geometry, size or dtype        */
#define CBCT_ERR_OOM -2       /* device allocation failed / can never fit     */
#define CBCT_ERR_DEVICE -3    /* HIP runtime error                            */
#define CBCT_ERR_BUSY -4      /* server queue full                            */
#define CBCT_ERR_NOT_FOUND -5 /* unknown ticket or patient                    */
#define CBCT_ERR_NUMERIC -6   /* non-finite value detected                    */

/* Thread-local description of the last failure on this thread ("" if none). */
const char *cbct_last_error(void);

/* Storage type of a projector operand. */
typedef enum { CBCT_F32 = 0, CBCT_BF16 = 1, CBCT_F16 = 2 } cbct_dtype;

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */

typedef struct {
    int32_t nx, ny, nz;    /* voxels per axis                                  */
    double vx, vy, vz;     /* voxel size [mm]                                  */
    int32_t nu, nv;        /* detector pixels (u across the orbit, v along z)  */
    double du, dv;         /* detector pitch [mm]                              */
    double dso, dsd;       /* source-isocentre, source-detector distance [mm]  */
    int32_t n_views;       /* projections                                      */
    const double *angles;  /* HOST array [n_views] in radians, copied; NULL =>
                              2*pi*k/n_views, k = 0..n_views-1                  */
} cbct_geom_desc;

typedef struct cbct_geom cbct_geom; /* opaque, immutable, shareable across threads */

/*
 * Create a geometry handle from a host descriptor (the projection geometry of
 * the linear model A x + e = b, paper Sec. 2.1, eq. "tomo").  Validates: all
 * sizes > 0; DSD > DSO; the source outside the volume's bounding sphere; the
 * detector beyond the volume; and a cone angle small enough that a ray moves
 * less than one voxel in z while it crosses one voxel column in x-y (at most
 * one z-plane per x-y cell; |cone half-angle| below about 35 degrees for cubic
 * voxels).  Device tables are built lazily per device at first use.
 * Errors: CBCT_ERR_INVALID (bad descriptor), CBCT_ERR_OOM (host allocation).
 */
int cbct_geom_create(const cbct_geom_desc *d, cbct_geom **out);
void cbct_geom_destroy(cbct_geom *g);
/* Number of voxels (M) and of projection samples (N = n_views * nv * nu). */
int cbct_geom_sizes(const cbct_geom *g, int64_t *n_vox, int64_t *n_proj);
/* Number of non-zero entries of A (ray/voxel pairs with positive chord), counted
 * on the device by the forward kernel's own traversal.  Synchronises
 * `hip_stream`.  Meant for reporting the algorithmic traffic of A and A^T. */
int cbct_geom_nnz(const cbct_geom *g, int64_t *nnz, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Projector pair                                                            */

/*
 * y = A x (overwrite): the sensing matrix of the linear CT model (paper Sec.
 * 2.1, eq. "tomo"), read as the exact chord length in mm of the ray from the
 * source to each pixel centre through each voxel.  x[z][y][x] holds dtype xt
 * with value = stored * x_scale; y[view][v][u] is float32.  FP32 accumulation.
 * Stream-ordered.  Temporary device memory (about 4*(M+N) bytes) is taken with
 * stream-ordered allocation on `hip_stream`.
 * Errors: CBCT_ERR_INVALID (null pointer, bad dtype/scale), CBCT_ERR_OOM,
 * CBCT_ERR_DEVICE.
 */
int cbct_forward(const cbct_geom *g, const void *x, cbct_dtype xt, float x_scale, float *y,
                 void *hip_stream);

/*
 * x = A^T y (overwrite): the literal transpose of cbct_forward's FP32 matrix
 * (Krylov methods need products with A and its transpose, paper Sec. 2.2.2).
 * The two kernels evaluate every chord with the same float32 operations, so
 * the pair is exactly adjoint up to summation order.  y[view][v][u] holds
 * dtype yt (value = stored * y_scale); x[z][y][x] float32.  Errors as
 * cbct_forward.
 */
int cbct_back(const cbct_geom *g, const void *y, cbct_dtype yt, float y_scale, float *x,
              void *hip_stream);

/*
 * Views per launch of A^T for geometry g (a tuning knob; 0 = automatic, the
 * default).  cbct_back, cbct_back_cols and the solvers run A^T as one launch per
 * chunk of consecutive views; each launch continues the cells' float32 partial
 * sums left in the output by the one before.  Short chunks keep the detector
 * data that the blocks resident on one XCD read within that XCD's L2; the
 * automatic choice bounds a 16 x 16-column square's detector footprint over a
 * chunk at about 3.5 MB.  Every chunk size gives the same results bit for bit.
 * Takes effect on the next call with g; not to be called while another thread
 * uses g.  Errors: CBCT_ERR_INVALID (null g, views < 0).
 */
int cbct_geom_set_back_views(cbct_geom *g, int views);

/*
 * Allocation-free cbct_forward, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operation, arguments, layouts and results as cbct_forward
 * (bit for bit: the same kernels), but its temporaries -- the padded column copy
 * of x (4 bytes per cell for CBCT_F32, 2 for BF16 / F16, pads and guards
 * included: (nz + 2) * nx * ny + 128 cells) and the column-layout projections
 * (4 * N bytes), each rounded up to 256 bytes -- live in one fixed device array
 * of the library of CBCT_FORWARD_NOALLOC_MAX_BYTES bytes per device.  That
 * array is placed on a device the first time this call runs there and is held
 * until the process ends.  The call allocates and frees nothing.
 * Preconditions: the geometry's tables must already be on the current device
 * (any earlier cbct_forward, cbct_back, solve or FDK call with g on this device
 * placed them), and the temporaries must fit the array; otherwise the call
 * returns CBCT_ERR_INVALID (with a message) before enqueueing anything.
 * Every call on one device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (different streams, or threads
 * without stream ordering between them) race and must not be issued.
 * Errors: CBCT_ERR_INVALID (null pointer, bad dtype/scale, size, tables not on
 * the device), CBCT_ERR_DEVICE.
 */
#define CBCT_FORWARD_NOALLOC_MAX_BYTES ((size_t)256 << 20)
int cbct_forward_noalloc(const cbct_geom *g, const void *x, cbct_dtype xt, float x_scale,
                         float *y, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Column layout (the kernels' native layout)                                */
/*
 * Callers that chain many products can keep data in the layouts the kernels
 * use and skip the transposes of cbct_forward / cbct_back:
 *  - column volume: a buffer of vol_floats floats; cell (i, j, k) lives at
 *    buf[vol_offset + (j*nx + i)*(nz + 2) + k + 1]; every other entry (one pad
 *    cell below and above each column, guards at both ends) must be zero;
 *  - column projections: ycols[view][u][v] (v fastest), proj_floats floats;
 *  - weighted column projections: L(u, v) * y, with L = |pixel - source| =
 *    sqrt(DSD^2 + u^2 + v^2) the ray length (the input of cbct_back_cols).
 */
int cbct_col_sizes(const cbct_geom *g, int64_t *vol_floats, int64_t *vol_offset,
                   int64_t *proj_floats);
/* x[z][y][x] -> column volume (writes every entry, pads and guards included). */
int cbct_vol_to_cols(const cbct_geom *g, const float *x, float *cols, void *hip_stream);
/* column volume -> x[z][y][x]. */
int cbct_cols_to_vol(const cbct_geom *g, const float *cols, float *x, void *hip_stream);
/* y[view][v][u] -> column projections; weighted != 0 multiplies by L(u, v). */
int cbct_proj_to_cols(const cbct_geom *g, const float *y, float *ycols, int weighted,
                      void *hip_stream);
/* column projections -> y[view][v][u]. */
int cbct_cols_to_proj(const cbct_geom *g, const float *ycols, float *y, void *hip_stream);
/* ycols = A x for a column volume (same kernel and chords as cbct_forward). */
int cbct_forward_cols(const cbct_geom *g, const float *cols, float *ycols, void *hip_stream);
/* cols = A^T y from weighted column projections (same kernel as cbct_back); pads and
 * guards of cols are written as zero. */
int cbct_back_cols(const cbct_geom *g, const float *ywcols, float *cols, void *hip_stream);

/*
 * TV reweighting (paper Sec. 2.2.1, definition of W~*, and Sec. 2.2.2 for the
 * PICCS pair): per voxel
 *   w1 = (sqrt(|D x|^2) + tau^2)^(-1/2),  w2 = (sqrt(|D x - D xp|^2) + tau^2)^(-1/2),
 * with D the forward differences x_i - x_{i+1} along x, y and z, zero at each
 * axis' last index (D_1 padded with a zero last row), and one weight per voxel
 * shared by the three directions.  All arrays x[z][y][x] float32, device.
 * Errors: CBCT_ERR_INVALID (null pointer, tau < 0), CBCT_ERR_OOM, CBCT_ERR_DEVICE.
 */
int piccs_weights(const cbct_geom *g, const float *x, const float *xp, double tau, float *w1,
                  float *w2, void *hip_stream);

/*
 * FDK reconstruction (Feldkamp, Davis & Kress 1984), the direct cone-beam
 * method of the clinical flow (Sec. 3 compares against it): a first image when
 * no prior exists.  y[view][v][u] line integrals -> x[z][y][x]:
 *   1. weight each sample by DSD / sqrt(DSD^2 + u^2 + v^2);
 *   2. convolve each detector row along u with the band-limited ramp filter at
 *      the isocentre pitch dp = du DSO / DSD;
 *   3. x(r) = sum over views of (dbeta/2) (DSO/U)^2 Q(u(r), v(r)), U the depth
 *      of r along the central ray, bilinear interpolation, zero outside the
 *      detector; dbeta is half the angle between a view's two neighbours on
 *      the circle (2 pi / V for equal spacing).
 * Full 360-degree scans.  Device pointers; a temporary of (N + M) floats is
 * taken from the stream's memory pool.  Errors: CBCT_ERR_INVALID (null pointer,
 * nu > 4680), CBCT_ERR_OOM, CBCT_ERR_DEVICE.
 */
int cbct_fdk(const cbct_geom *g, const float *y, float *x, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* IRN-PICCS Krylov solve                                                    */

typedef enum {
    CBCT_PREC_FP32 = 0,       /* float32 storage and projector arithmetic           */
    CBCT_PREC_MIXED_BF16 = 1, /* bf16 operand of A (the LSQR vector v), fp32         */
                              /* accumulation; A^T reads float32                    */
    CBCT_PREC_MIXED_F16 = 2,  /* scaled fp16 operand of A, fp32 accumulation         */
    CBCT_PREC_MIXED_BF16_ADJ16 = 3, /* as MIXED_BF16, and A^T reads a bf16 copy of   */
                                    /* its operand u-hat as well                     */
    CBCT_PREC_MIXED_F16_ADJ16 = 4   /* as MIXED_F16, and A^T reads a scaled fp16     */
                                    /* copy of u-hat as well                         */
} cbct_precision;

/* The prior term (Sec. 2.1): PICCS penalises TV(x - x_p) (eq. "PICCS problem",
 * third block lambda W2 D, right-hand side lambda W2 D x_p); PIPLE penalises
 * ||x - x_p||_2^2 (eq. "PIRPLE_problem", solved by eq. "seq_W_2": third block
 * lambda I, right-hand side lambda x_p; W2 is not used). */
typedef enum { CBCT_METHOD_PICCS = 0, CBCT_METHOD_PIPLE = 1 } cbct_method;

typedef struct {
    double alpha;     /* weight of TV(x)           (paper eq. "PICCS problem")   */
    double lambda;    /* weight of TV(x - x_p)                                    */
    double tau;       /* smoothing of the TV weights (Sec. 2.2.1)                  */
    int32_t n_outer;  /* IRN reweightings                                         */
    int32_t n_inner;  /* LSQR iterations per reweighting (total = outer * inner)  */
    int32_t precision;/* cbct_precision                                           */
    int32_t reorth;   /* 0: none (the paper's short recurrences); 1: one-sided     */
                      /* reorthogonalisation of v: classical Gram-Schmidt twice   */
                      /* against this outer step's v's, float64 arithmetic; adds  */
                      /* n_inner volumes to the workspace (not in the paper)      */
    int32_t method;   /* cbct_method: which prior term the third block encodes     */
} piccs_params;

typedef struct {
    int32_t inner_done;  /* LSQR iterations actually performed (all outers)          */
    int32_t outer_done;  /* reweightings performed                                     */
    int32_t breakdown;   /* number of inner solves that stopped on beta or alpha = 0   */
    double *resid_hist;  /* optional HOST array [n_outer*n_inner] receiving LSQR's
                            phi-bar (= ||b~ - A~ x||) after every inner iteration, or NULL */
} piccs_report;

/* Device workspace needed by piccs_krylov_solve for this geometry and params. */
int piccs_workspace_bytes(const cbct_geom *g, const piccs_params *p, size_t *bytes);

/*
 * IRN-PICCS (paper Sec. 2.2.2, eq. "PICCS_rec" and the augmented least-squares
 * problem): for k = 1..n_outer, W1 = W~(D x_{k-1}), W2 = W~(D x_{k-1} - D x_p),
 * then n_inner LSQR iterations (Paige & Saunders 1982) on
 *   [A; alpha W1 D; lambda W2 D] x ~ [b; 0; lambda W2 D x_p]
 * restarted from x_{k-1}.  With p->method = CBCT_METHOD_PIPLE the third block is
 * lambda I with right-hand side lambda x_p (IRN-PIPLE, Sec. 2.2.1, eq. "seq_W_2").
 * lambda = 0 gives IRN-TV and alpha = lambda = 0 plain least squares.  The
 * LSQR scalars (norms, Givens rotation) are kept in FP64 on the device; the
 * host never waits inside the solve.  p->reorth = 1 adds a one-sided
 * reorthogonalisation of v (not in the paper; see piccs_params).
 * b[view][v][u], xp and x[z][y][x] are float32 device arrays; x holds x_0 on
 * entry (warm start) and x_K on return.  workspace: >= piccs_workspace_bytes,
 * device, 256-byte aligned.  If rep != NULL the call synchronises the stream
 * and fills the report; otherwise it returns after enqueueing.
 * A norm that comes out non-finite (NaN or Inf in b, x_0 or x_p, or an
 * overflow) stops the solve at that point, leaving the last finite iterate in
 * x; with rep != NULL the call then returns CBCT_ERR_NUMERIC (the report is
 * filled first).
 * Errors: CBCT_ERR_INVALID, CBCT_ERR_DEVICE, CBCT_ERR_NUMERIC.
 */
int piccs_krylov_solve(const cbct_geom *g, const float *b, const float *xp, float *x,
                       const piccs_params *p, void *workspace, size_t ws_bytes,
                       piccs_report *rep, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of repeated-scan reconstructions             */
/*
 * The paper motivates the method by repeated scans of one patient during an
 * intervention, each reconstructed from few views against a prior image
 * (Sec. 1 and Sec. 2.2.2).  A server runs such requests for many patients on
 * one device:
 *  - every request is one IRN-PICCS solve (piccs_krylov_solve) of its own
 *    geometry and parameters against its patient's prior;
 *  - each patient's prior x_p and previous reconstruction x_prev stay
 *    resident on the device; a request starts from x_prev (warm start) or
 *    from x_p;
 *  - requests are admitted in arrival order as stream slots and HBM budget
 *    free up, and admitted requests run concurrently on their own streams;
 *    requests of one patient run one at a time in arrival order;
 *  - the budget covers everything the server places on the device: residents
 *    (8 bytes per voxel per patient), cached projector tables of each
 *    geometry, and per running request b, x and the solve workspace.
 * All server calls are thread-safe.  Times are seconds on a monotonic clock
 * since cbct_server_create.
 */
typedef struct {
    size_t hbm_budget_bytes; /* device memory the server may use; 0 = 90 % of free  */
    int32_t max_slots;       /* concurrent requests on the device (streams), >= 1    */
    int32_t device;          /* HIP device ordinal                                   */
    int32_t max_queue;       /* waiting requests before CBCT_ERR_BUSY; 0 = 4096      */
} cbct_server_config;

typedef struct cbct_server cbct_server;

typedef enum {
    CBCT_X0_PREVIOUS = 0, /* start from the patient's last reconstruction, else x_p */
    CBCT_X0_PRIOR = 1     /* start from x_p                                          */
} cbct_x0_source;

typedef struct {
    int32_t patient;       /* id given to cbct_server_add_prior                     */
    cbct_geom_desc geom;   /* scan geometry; its volume must be the patient's       */
    const float *b_host;   /* HOST projections b[view][v][u]; copied at submit      */
    piccs_params params;   /* solve parameters                                      */
    int32_t x0;            /* cbct_x0_source                                        */
} cbct_request;

typedef struct {
    int32_t status;        /* CBCT_OK or the request's error (CBCT_ERR_NUMERIC: a non-
                              finite norm, e.g. NaN or Inf in b or the start image)  */
    double t_submit;       /* submit returned                                        */
    double t_admit;        /* admitted: its work was enqueued on the device          */
    double t_done;         /* result ready to poll                                   */
    piccs_report report;   /* set report.resid_hist (HOST, n_outer*n_inner) before
                              polling to receive the residual history               */
} cbct_result;

typedef struct {
    int64_t capacity, used, peak_used, resident; /* bytes of the HBM budget          */
    int64_t queued, in_flight, peak_in_flight, done_unpolled;
    int64_t completed, failed, geom_placements, geom_evictions;
} cbct_server_stats;

/* Reserves the budget on the device and starts the scheduler thread.
 * Errors: CBCT_ERR_INVALID (max_slots < 1, bad device), CBCT_ERR_OOM. */
int cbct_server_create(const cbct_server_config *c, cbct_server **out);

/* Registers patient `patient` with prior image xp_host[z][y][x] (HOST, copied;
 * the call returns once it is on the device).  The volume of g is the
 * patient's volume.  Errors: CBCT_ERR_INVALID (bad geometry, id already
 * registered), CBCT_ERR_OOM (residents do not fit in the budget). */
int cbct_server_add_prior(cbct_server *s, int32_t patient, const cbct_geom_desc *g,
                          const float *xp_host);

/* Queues a request and returns at once with its ticket (> 0).  Errors:
 * CBCT_ERR_INVALID (geometry, volume mismatch, params), CBCT_ERR_NOT_FOUND
 * (unknown patient), CBCT_ERR_BUSY (queue full), CBCT_ERR_OOM (the request
 * cannot fit beside the residents even on an idle device). */
int cbct_server_submit(cbct_server *s, const cbct_request *r, uint64_t *ticket);

/* Non-blocking.  CBCT_PENDING while the request is queued or running;
 * CBCT_ERR_NOT_FOUND for an unknown or already collected ticket.  Once
 * finished, copies x[z][y][x] into x_host_out (HOST, may be NULL), fills *res
 * (may be NULL), forgets the ticket and returns the request's status. */
int cbct_server_poll(cbct_server *s, uint64_t ticket, float *x_host_out, cbct_result *res);

/* Device bytes the server needs (host-only computation, no device access):
 * *request_bytes while a request of this geometry and params runs (b, x and
 * the solve workspace), *tables_bytes for the geometry's cached projector
 * tables, *resident_bytes per patient of this volume (x_p and x_prev).  Any
 * output pointer may be NULL.  Errors: CBCT_ERR_INVALID. */
int cbct_server_footprint(const cbct_geom_desc *g, const piccs_params *p, size_t *request_bytes,
                          size_t *tables_bytes, size_t *resident_bytes);

/* Snapshot of the scheduler's counters. */
int cbct_server_stats_get(cbct_server *s, cbct_server_stats *out);

/* Waits for every queued and running request to finish, then releases the
 * device memory, streams and thread.  Results never polled are dropped. */
int cbct_server_destroy(cbct_server *s);

#ifdef __cplusplus
}
#endif
#endif /* CBCT_H */
