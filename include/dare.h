/*
 * dare.h -- C ABI of the MI355X (gfx950) directionality-aware ultrasound
 * reconstruction and reslicing library.
 *
 * Method: "Real-time, Directionality Aware 3D Ultrasound Reconstruction and
 * Re-Slicing" (DARE), Sec. 2.1.  Tracked 2D frames are voxelized into a grid
 * that keeps, per voxel, what was seen from each acquisition direction
 * ("Volume reconstruction", Fig. 1); a virtual plane at any pose is then
 * resliced by gathering each pixel's cubic neighbourhood, discarding samples
 * whose direction is misaligned beyond two angular thresholds and blending
 * the rest with the exponential weights of Eq. 1 and Eq. 2, weighted by
 * distance (Fig. 2); a pixel with no surviving sample is unassigned.
 *
 * Conventions shared by every entry point:
 *   - Millimetres everywhere.  4x4 poses are row-major; the last row is
 *     (0, 0, 0, 1).  A *probe pose* maps probe coordinates to world (what the
 *     tracker reports); the calibration maps image millimetres to the probe,
 *     so an image's pose is T = P . C.  Column 0 of T is the lateral (x)
 *     axis, column 1 the depth (beam) axis, column 2 the plane normal.
 *   - Pixel (i, j) of a frame or slice is column i (lateral), row j (depth);
 *     it lies at image millimetres (i * pitch[0], j * pitch[1], 0).  Images
 *     are row-major, row j at offset j * width.
 *   - Voxel (ix, iy, iz) has its centre at origin + spacing * (ix, iy, iz).
 *   - Pose composition and sample positions are evaluated in FP64 on the GPU,
 *     without fused multiply-add and in a fixed order, so that nearest-voxel
 *     decisions are reproducible bit for bit.
 *   - "_dev" pointers are device memory of the current HIP device; host
 *     structs are read before the call returns.  Every call that takes a
 *     stream is asynchronous on it unless documented otherwise; device
 *     buffers must stay valid until the stream reaches the call.
 *   - Errors are status codes; no exception crosses the ABI.  On any error
 *     other than DARE_WARN_BINS_SATURATED nothing has been enqueued, or the
 *     volume has been restored to its state before the call.
 *   - A `stream` argument is a hipStream_t passed as void*; NULL is the
 *     default stream.
 */
#ifndef DARE_H
#define DARE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DARE_OK = 0,
    DARE_ERR_INVALID_ARG = 1,     /* null pointer, size <= 0, unsupported radius or dtype     */
    DARE_ERR_BAD_POSE = 2,        /* non-finite pose, or rotation with |R^T R - I|_inf > 1e-4 */
    DARE_ERR_BUDGET = 3,          /* the volume's arena cannot hold the new bricks            */
    DARE_ERR_HIP = 4,             /* a HIP runtime call failed                                */
    DARE_WARN_BINS_SATURATED = 5, /* codebook full: frames went to their closest bin         */
    DARE_ERR_NOT_READY = 6,       /* server ticket still in flight                            */
    DARE_ERR_QUEUE_FULL = 7       /* server admission queue is full                           */
} dare_status;

/* Storage precision of the directional grid (values and counts).  The
 * reslice accumulates in FP32 whatever the storage; poses and positions are
 * always FP64.  FP8 is OCP e4m3fn with one FP32 scale per (bin, brick) for
 * the values and one for the counts. */
typedef enum { DARE_F32 = 0, DARE_BF16 = 1, DARE_F16 = 2, DARE_FP8_E4M3 = 3 } dare_dtype;

/* Volume geometry (Sec. 2.1: "a 3D bounding box ... voxelized into a 3D grid"). */
typedef struct {
    double origin_mm[3];   /* world position of voxel (0,0,0)'s centre                     */
    double spacing_mm;     /* isotropic voxel size h > 0                                    */
    int32_t dims[3];       /* nx, ny, nz > 0                                                */
    double calib[16];      /* image-mm -> probe, row-major (the probe calibration)          */
} dare_geometry;

/* Method parameters.  Defaults (dare_default_params): k_normal = 10,
 * k_inplane = 5, thresholds 25 and 15 degrees (Sec. 2.1, constants after
 * Eq. 2); radius_vox = 1 (interpolation distance of one voxel, the paper's
 * 0.125 mm at 0.125 mm voxels); bin_tol_deg = 5 and max_bins = 64 for the
 * codebook of acquisition orientations; normal_axis = 2 (the acquisition
 * normal of Eq. 1 is the image-plane normal; 1 selects the beam axis). */
typedef struct {
    double k_normal, k_inplane;
    double thr_normal_deg, thr_inplane_deg;
    double radius_vox;     /* R: integer 1..8; the neighbourhood is |c - v|_inf < R         */
    double bin_tol_deg;    /* leader-clustering tolerance delta, degrees, >= 0              */
    int32_t max_bins;      /* 1..64                                                         */
    int32_t normal_axis;   /* 1 or 2                                                        */
} dare_params;

/* A reslice request: the virtual image plane of Sec. 2.1 "Reslicing". */
typedef struct {
    double probe_pose[16]; /* probe -> world, row-major, FP64                               */
    int32_t width, height; /* output pixels, > 0                                            */
    double pitch_mm[2];    /* pixel spacing along the lateral and depth axes, > 0           */
} dare_slice_spec;

typedef struct dare_volume dare_volume;

typedef struct {
    int32_t bins;             /* codebook size K                                         */
    int32_t saturated;        /* 1 once a frame could not open a new bin                 */
    int64_t bricks_used;      /* allocated (bin, 8^3 brick) slots                        */
    int64_t bricks_capacity;  /* slots the arena can hold                                */
    int64_t bytes_per_brick;  /* accumulators + stored pairs (+ scales) per slot         */
    int64_t brick_grid[3];    /* bricks along x, y, z                                    */
} dare_volume_info;

/* Fill *p with the paper's parameters (see dare_params). */
void dare_default_params(dare_params* p);

/* Text of a status code (static storage). */
const char* dare_status_str(dare_status s);

/* Bytes of arena a volume needs for `bricks` allocated (bin, brick) slots,
 * including its fixed tables.  Use it to size `arena_bytes`. */
uint64_t dare_volume_arena_bytes(const dare_geometry* g, const dare_params* p, dare_dtype dtype,
                                 int64_t bricks);

/* Create an empty volume whose whole device state lives in the caller's
 * arena [arena_dev, arena_dev + arena_bytes) on the current device; the
 * arena size is the volume's HBM budget.  The arena must stay allocated
 * until dare_volume_destroy.  Synchronous.  Errors: INVALID_ARG (null,
 * non-positive dims/spacing, bad params, arena without room for the fixed
 * tables and one brick slot), BAD_POSE (calibration not rigid), HIP. */
dare_status dare_volume_create(const dare_geometry* g, const dare_params* p, dare_dtype dtype,
                               void* arena_dev, uint64_t arena_bytes, dare_volume** out);

/* Release the handle (not the arena).  Synchronises the device first. */
dare_status dare_volume_destroy(dare_volume* v);

/* Volume reconstruction (Sec. 2.1, Fig. 1): compose each frame's pose with
 * the calibration, assign it to a direction bin, voxelize every pixel to its
 * nearest voxel (ties rounded up) and add its intensity and a count to that
 * (bin, voxel); pixels outside the grid are dropped.  Frames are added to
 * what the volume already holds (incremental), in the given order.
 *   frames_dev       n * h * w uint8, frame-major, row-major images
 *   probe_poses_dev  n * 16 float32, row-major probe poses
 *   pitch_mm         pixel spacing of the frames (host)
 * Sums are exact integers, so the result does not depend on thread order.
 * Synchronises `stream` once per batch of up to 4096 frames (pose check and
 * budget admission); the final finalize step is left enqueued.
 * Errors: INVALID_ARG, BAD_POSE (a frame pose is not rigid: that batch is
 * rolled back), BUDGET (the new bricks do not fit: that batch is rolled
 * back), HIP.  Returns DARE_WARN_BINS_SATURATED when the codebook is full. */
dare_status dare_reconstruct_frames(dare_volume* v, const uint8_t* frames_dev, int32_t n, int32_t w,
                                    int32_t h, const double pitch_mm[2], const float* probe_poses_dev,
                                    void* stream);

/* Fan probes: curvilinear arrays, and phased arrays (r0_mm = 0).  The paper
 * images with a linear array (Sec. 2.2), whose samples all share the frame's
 * in-plane direction, the x-axis Eq. 1 compares.  A fan's beams leave one
 * apex at different angles, so that direction changes across the columns:
 * column i's beam has unit direction b_i = (b_i0, b_i1) in image millimetres
 * (lateral, axial), and pixel (i, j) lies on it at r = r0 + j * dr from the
 * apex a, at image millimetres (a0 + r b_i0, a1 + r b_i1), placed in the
 * world as a linear-array pixel at those millimetres.  Its in-plane direction
 * is the one across its beam, b_i1 xhat - b_i0 yhat (xhat, yhat: the image
 * axes in the world).  Binning per column fan: the columns are split into
 * `sectors` equal sectors (column i in sector i * sectors / w), each sector's
 * samples taking the in-plane direction of its middle column, and every
 * (frame, sector) enters the direction binning as a frame of its own, frames
 * in order, sectors in order.  Reslicing is unchanged. */
typedef struct {
    double apex_mm[2];     /* the fan's apex, image mm (lateral, axial), finite */
    double r0_mm;          /* distance of the first row from the apex, >= 0     */
    double dr_mm;          /* radial step per row, > 0                          */
    int32_t sectors;       /* 1 .. min(64, w)                                    */
} dare_fan;

/* Volume reconstruction from fan frames: dare_reconstruct_frames with the
 * pixel placement and per-sector binning above.
 *   beams_dev  w * 2 doubles on the device: every column's unit beam
 *              direction (not checked; the caller's table is used as given).
 * The volume's normal_axis must be 2 (the image-plane normal): INVALID_ARG
 * otherwise.  Batches hold 4096 / sectors frames.  Errors and return values as
 * dare_reconstruct_frames. */
dare_status dare_reconstruct_fan(dare_volume* v, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                                 const dare_fan* fan, const double* beams_dev, const float* probe_poses_dev,
                                 void* stream);

/* Reslice one plane (Sec. 2.1 "Reslicing", Eq. 1, Eq. 2): the slice pose
 * composed with the calibration in FP64 on the device, Eq. 1 for every bin of
 * the codebook, both angular thresholds and Eq. 2 for the survivors (FP64 on
 * the device); then for each output pixel the FP64 sample position, its
 * neighbourhood |c - v|_inf < R with tent weights prod(1 - |c_a - v_a| / R),
 * per-voxel direction blending with the angular weight of each surviving bin,
 * and the distance-weighted average over valid voxels.
 *   out_dev   height * width float32, row-major; NaN marks an unassigned pixel.
 * Enqueues a single kernel; allocates nothing.  Errors: INVALID_ARG,
 * BAD_POSE (slice pose not rigid), HIP. */
dare_status dare_reslice(const dare_volume* v, const dare_slice_spec* spec, float* out_dev, void* stream);

/* Bytes of device workspace dare_reslice_batch needs for these n requests. */
uint64_t dare_reslice_batch_workspace_bytes(const dare_volume* const* vols, const dare_slice_spec* specs,
                                            int32_t n);

/* Reslice n planes, possibly of different volumes, sizes and poses, in one
 * launch sequence per (storage dtype, radius) group; a group holds at most
 * 4096 requests, taken in call order (more make further groups).  Each
 * request's result equals what dare_reslice gives for it alone.
 *   vols       n volume handles (host array)
 *   specs      n requests (host array)
 *   outs_dev   n device output pointers (host array), each height*width float32
 *   workspace_dev / workspace_bytes: device scratch for the request table,
 *              at least dare_reslice_batch_workspace_bytes; must not be in use
 *              by another in-flight call.
 * Errors: INVALID_ARG, BAD_POSE, HIP. */
dare_status dare_reslice_batch(const dare_volume* const* vols, const dare_slice_spec* specs,
                               float* const* outs_dev, int32_t n, void* workspace_dev,
                               uint64_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): dare_reslice_batch
 * with its workspace in a device buffer the library holds, of
 * DARE_NOALLOC_WORKSPACE_BYTES on each device it runs on, kept until the
 * process ends (its address is taken once per device, on the first call there).
 * The call allocates nothing; the request table is copied from pageable host
 * memory, so the call returns once the copy has read it.  Every call on a device
 * shares that device's buffer: calls that overlap on one device (other streams,
 * other threads) race and must not be issued; successive calls on one stream
 * are safe.  Results are those of dare_reslice_batch, bit for bit.
 * Errors: as dare_reslice_batch; BUDGET (nothing launched) when the batch needs
 * more than DARE_NOALLOC_WORKSPACE_BYTES of workspace (see
 * dare_reslice_batch_workspace_bytes). */
#define DARE_NOALLOC_WORKSPACE_BYTES (32ull << 20)
dare_status dare_reslice_batch_noalloc(const dare_volume* const* vols, const dare_slice_spec* specs,
                                       float* const* outs_dev, int32_t n, void* stream);

/* Bounding box of the frames (Sec. 2.1: computed from the collected
 * transducer positions): the axis-aligned box of every frame's four corner
 * pixel centres, origin = its minimum corner, dims = ceil(extent / h) + 1.
 * Host-only.  probe_poses_host: n * 16 float32.  Copies the calibration into
 * out->calib.  Errors: INVALID_ARG, BAD_POSE. */
dare_status dare_bounds_from_frames(const float* probe_poses_host, int32_t n, int32_t w, int32_t h,
                                    const double pitch_mm[2], const double calib[16], double spacing_mm,
                                    dare_geometry* out);

/* Volume bookkeeping.  Synchronises the device. */
dare_status dare_volume_get_info(const dare_volume* v, dare_volume_info* out);

/* Codebook readback: up to 64 representative (normal, x-axis) unit vectors,
 * 3 doubles each, and the bin count.  Synchronises the device. */
dare_status dare_volume_get_codebook(const dare_volume* v, double* rep_n_host, double* rep_x_host,
                                     int32_t* bins);

/* Dense copies for tests and tools.  All arrays are (bins, nz, ny, nx),
 * x fastest, on the device; `bins` must equal the volume's bin count.
 *   download_sums:    exact per-(bin, voxel) intensity sums and counts.
 *   download_storage: the stored values and counts as the reslice reads them
 *                     (dequantised to float32), 0 where the voxel is empty.
 *   upload_sums:      replace the volume's content with given sums/counts and
 *                     codebook (rep arrays: bins * 3 doubles, host), then
 *                     finalize; BUDGET if the occupied bricks do not fit.
 * upload synchronises the stream; the downloads are asynchronous. */
dare_status dare_volume_download_sums(const dare_volume* v, uint32_t* sums_dev, uint32_t* counts_dev,
                                      int32_t bins, void* stream);
dare_status dare_volume_download_storage(const dare_volume* v, float* values_dev, float* counts_dev,
                                         int32_t bins, void* stream);
dare_status dare_volume_upload_sums(dare_volume* v, const double* rep_n_host, const double* rep_x_host,
                                    int32_t bins, const uint32_t* sums_dev, const uint32_t* counts_dev,
                                    void* stream);

/* Volume persistence: save a volume's whole state (geometry, parameters,
 * dtype, codebook, brick table, exact accumulators, stored pairs and FP8
 * scales) to host memory, and load it into a new arena, possibly on another
 * device or process.  A loaded volume reslices bit for bit like the saved one
 * and keeps compounding incrementally (the accumulators travel with it).
 * The format is this library's own (a versioned header, then the arrays).
 *   save_bytes: bytes dare_volume_save writes (0 for an invalid handle).
 *   save:       synchronises the device; INVALID_ARG if bytes is too small
 *               or the volume holds bricks in host memory (restore them
 *               first: dare_volume_restore_box).
 *   load:       creates the volume in [arena_dev, arena_dev + arena_bytes)
 *               on the current device (as dare_volume_create) and fills it;
 *               INVALID_ARG for a damaged or foreign buffer, BUDGET if the
 *               arena cannot hold the saved bricks.  Synchronous.  The brick
 *               table is checked on the host before anything is uploaded:
 *               every entry -1 or a slot below the saved slot count, each such
 *               slot owned by exactly one entry, no entry in the rows of bins
 *               beyond the codebook, finite representatives; a table that
 *               breaks any of these is INVALID_ARG (no device call made). */
uint64_t dare_volume_save_bytes(const dare_volume* v);
dare_status dare_volume_save(const dare_volume* v, void* host_out, uint64_t bytes);
dare_status dare_volume_load(const void* host_in, uint64_t bytes, void* arena_dev, uint64_t arena_bytes,
                             dare_volume** out);

/* Out-of-core bricks (Sec. 4 names data sets beyond GPU memory and the
 * incremental integration of frames during a scan as the next steps).  A
 * (bin, 8^3 brick) can be moved to host memory ("held"): its exact
 * accumulators leave, its pool slot is freed, and reslices see the volume
 * without it.  Compounding carries on as usual: a frame that reaches a held
 * brick starts it afresh in HBM, and bringing the held part back adds the two
 * (integer sums) and refinalises.  Hence, once every held brick is restored,
 * the volume equals bit for bit the one a large enough arena would have
 * built, whatever was moved out and back, and when.  The host memory is the
 * library's and goes with dare_volume_destroy (or dare_volume_upload_sums).
 *   evict_outside: hold every resident brick that does not meet the voxel box
 *                  lo..hi (inclusive, voxel indices; lo > hi on an axis holds
 *                  every brick).  The pool is compacted.
 *   restore_box:   bring back every held brick that meets the box.  BUDGET,
 *                  with nothing changed, if the pool lacks free slots for the
 *                  ones not resident meanwhile.
 *   set_spill:     enabled != 0: a frame batch whose new bricks do not fit
 *                  first holds the least recently touched bricks (none that
 *                  the batch touches): enough for the batch and a sixteenth
 *                  of the pool more.  BUDGET remains for a batch that alone
 *                  touches more bricks than the pool has slots.  Off at
 *                  creation.
 *   held:          number of held bricks and the host bytes they take.
 * evict_outside and restore_box synchronise `stream`; none may overlap
 * another call on the same volume.  Errors: INVALID_ARG, BUDGET, HIP. */
dare_status dare_volume_evict_outside(dare_volume* v, const int32_t lo[3], const int32_t hi[3], void* stream);
dare_status dare_volume_restore_box(dare_volume* v, const int32_t lo[3], const int32_t hi[3], void* stream);
dare_status dare_volume_set_spill(dare_volume* v, int32_t enabled);
dare_status dare_volume_held(const dare_volume* v, int64_t* bricks, uint64_t* bytes);

/* The direction bins that survive both thresholds for this slice pose and
 * their Eq. 2 weights (Sec. 2.1, Eq. 1 and Eq. 2), evaluated on the host in
 * FP64 from the volume's codebook: a query for callers (and for counting a
 * slice's compulsory bytes); the reslices evaluate the same on the device.  bins_out / weights_out (may be NULL)
 * receive up to 64 entries; *count the number.  Synchronises the device.
 * Errors: INVALID_ARG, BAD_POSE, HIP. */
dare_status dare_slice_active_bins(const dare_volume* v, const dare_slice_spec* spec, int32_t* bins_out,
                                   double* weights_out, int32_t* count);

/* ------------------------------------------------------------------------
 * Per-sample store: Sec. 2.1 read literally (Fig. 1: every grid location
 * points into a flat store of the samples that landed there, each with its
 * own acquisition orientation; "Reslicing": every sample weighed by Eq. 1,
 * the two thresholds and Eq. 2 with its own frame's orientation).  No
 * direction bins: this is the formulation the binned volume approximates
 * (with bin_tol_deg = 0 and the tent reading the two agree), at GPU speed.
 * A store lives in a caller-supplied arena on the current device.
 * ------------------------------------------------------------------------ */
typedef struct dare_samples dare_samples;

/* Reslice readings of the per-sample store, for output position c and radius R:
 *   BOX   the (2R+1)^3 voxels around the nearest voxel floor(c + 0.5), one
 *         weighted average over all their samples: sum w I / sum w;
 *   TENT  the voxels with |c - v|_inf < R, each averaged over its samples
 *         (sum w I / sum w), then averaged with tent weights
 *         prod(1 - |c_a - v_a| / R) over the voxels with weight (the
 *         reading dare_reslice uses).
 * A pixel whose neighbourhood holds no sample of positive weight is NaN. */
typedef enum { DARE_LITERAL_BOX = 0, DARE_LITERAL_TENT = 1 } dare_literal_mode;

/* Arena bytes for a store over geometry g holding up to max_samples samples
 * (every in-grid frame pixel is one) from up to max_frames frames; 0 for
 * invalid arguments. */
uint64_t dare_samples_arena_bytes(const dare_geometry* g, int64_t max_samples, int32_t max_frames);
/* Create an empty store in [arena_dev, arena_dev + arena_bytes) (256-byte
 * aligned, kept allocated until destroy).  max_samples <= 2^32 - 1,
 * 1 <= max_frames <= 2^24.  Synchronous.  Errors: INVALID_ARG, BAD_POSE
 * (calibration not rigid), HIP. */
dare_status dare_samples_create(const dare_geometry* g, int64_t max_samples, int32_t max_frames, void* arena_dev,
                                uint64_t arena_bytes, dare_samples** out);
/* Release the handle (not the arena).  Synchronises the device first. */
dare_status dare_samples_destroy(dare_samples* s);
/* Replace the store's content with the samples of n frames: every pixel's
 * nearest voxel (floor(c + 0.5), positions as for dare_reconstruct_frames),
 * kept with its intensity and frame; pixels outside the grid are dropped.
 * The frames' acquisition normal is column normal_axis (1 or 2) of
 * T = P . C.  frames_dev: n * h * w uint8; probe_poses_dev: n * 16 float32,
 * row-major.  Synchronises `stream` twice (pose check, sample count); the
 * placing pass is left enqueued.  Errors: INVALID_ARG (n > max_frames),
 * BAD_POSE, BUDGET (more samples than max_samples), HIP; on any error the
 * store is left empty. */
dare_status dare_samples_build(dare_samples* s, const uint8_t* frames_dev, int32_t n, int32_t w, int32_t h,
                               const double pitch_mm[2], const float* probe_poses_dev, int32_t normal_axis,
                               void* stream);
/* Samples and frames the last build stored (host bookkeeping, no sync). */
dare_status dare_samples_count(const dare_samples* s, int64_t* n_samples, int32_t* n_frames);
/* Reslice one plane from the store in the given reading (dare_literal_mode)
 * with parameters p (radius_vox, thresholds, k_normal, k_inplane;
 * normal_axis must equal the build's): a per-frame weight table for the
 * slice, then one kernel over the output pixels.  out_dev: height * width
 * float32, row-major, NaN where unassigned.  Calls on one store must not
 * overlap in time (they share the weight table).  Errors: INVALID_ARG,
 * BAD_POSE, HIP. */
dare_status dare_samples_reslice(const dare_samples* s, const dare_params* p, const dare_slice_spec* spec,
                                 int32_t mode, float* out_dev, void* stream);

/* Image similarity of a reslice against the acquired frame at the same pose
 * (Sec. 3, quantitative evaluation: normalised cross-correlation and the
 * structural similarity index against ground truth).  Readings (the paper
 * names the measures only): zero-mean NCC over the pixels the reslice
 * assigns (finite); SSIM of Wang et al. with an 11 x 11 Gaussian window
 * (sigma 1.5, weights summing to 1), K1 = 0.01, K2 = 0.03, L = 255, averaged
 * over the pixels whose whole window lies inside the image and is assigned.
 *   image_dev  h * w float32 reslice (NaN = unassigned); frame_dev h * w uint8
 *   workspace_dev / workspace_bytes: device scratch, at least
 *              dare_compare_workspace_bytes(), 8-byte aligned
 *   out_host   4 doubles: NCC, mean SSIM (NaN when undefined), pixels used
 *              for NCC, windows used for SSIM.
 * Synchronises `stream`.  Errors: INVALID_ARG, HIP. */
uint64_t dare_compare_workspace_bytes(void);
dare_status dare_compare_to_frame(const float* image_dev, const uint8_t* frame_dev, int32_t w, int32_t h,
                                  void* workspace_dev, uint64_t workspace_bytes, double* out_host, void* stream);

/* Streaming copy of n_bytes (multiple of 16) from src_dev to dst_dev: the
 * bandwidth probe that calibrates the HBM roofline and the byte counters. */
dare_status dare_copy_probe(const void* src_dev, void* dst_dev, uint64_t n_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of reslice requests from many consoles (the
 * expert consoles of Sec. 1 each reslice the shared volume at their own
 * pose).  A server owns a caller-supplied device arena (the HBM budget of its
 * results: one workspace per stream, laid out when the first volume is added,
 * and the result slots), up to `n_streams` (1..4) HIP streams of default
 * priority, and a host thread that groups waiting requests into ticks.  A
 * request is admitted, first come first served, when a result slot of its
 * size can be allocated in the arena; each tick uploads its request table,
 * replays a captured graph of the batched reslice on a free stream (ticks on
 * different streams overlap on the device), then copies every result into its
 * `host_out` buffer (pinned host memory keeps the copy asynchronous; a device
 * buffer on the server's GPU keeps the result there, with no transfer over
 * the host link).
 * Volumes are admitted against a second budget, `volume_budget_bytes`: the
 * device bytes of the resident volumes' arenas (Sec. 4 names dataset size
 * against GPU memory as the limit to plan for); a removed volume returns its
 * bytes.  All volumes of one server share one storage dtype and radius.
 * Volumes must not be reconstructed while the server can reslice them.
 * ------------------------------------------------------------------------ */
typedef struct dare_server dare_server;

typedef struct {
    int64_t max_tick_pixels;  /* pixels per tick (bounds one launch); >= largest request, <= 2^32 */
    int32_t max_tick_requests;/* requests per tick, 1..4096                                 */
    int32_t n_streams;        /* 1..4                                                        */
    int32_t max_queue;        /* waiting requests before submit returns QUEUE_FULL          */
    int32_t use_graphs;       /* 1: replay captured graphs per tick; 0: plain launches       */
    uint64_t volume_budget_bytes; /* device bytes of resident volumes' arenas; 0 = no limit   */
} dare_server_config;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t ticks;
    int64_t pixels;
    double busy_seconds;      /* host-measured time with at least one tick in flight         */
    int64_t frames;           /* frames compounded through dare_server_submit_frames         */
    double compound_seconds;  /* host-measured time spent compounding them                   */
    double kernel_seconds;    /* device-measured: sum over ticks of the span of their kernels */
    double device_busy_seconds; /* device-measured: union of those spans (ticks on different
                                   streams overlap), i.e. time the device ran served kernels  */
    int64_t untimed_ticks;    /* ticks whose kernel span could not be read (not in the above) */
} dare_server_stats;

typedef struct {
    double t_submit, t_admit, t_launch, t_device_done, t_host_done; /* seconds, steady clock */
} dare_request_times;

/* Defaults: 8 Mpixel and 64 requests per tick, 3 streams, 4096 queued, graphs on, no volume
 * budget. */
void dare_default_server_config(dare_server_config* c);
/* arena_dev: 256-byte aligned device memory of at least 512 bytes, kept allocated until
 * destroy. */
dare_status dare_server_create(const dare_server_config* cfg, void* arena_dev, uint64_t arena_bytes,
                               dare_server** out);
/* Register a volume (it stays owned by the caller).  INVALID_ARG if its dtype or radius
 * differs from the first one's, if it lives on another device or is registered already;
 * BUDGET if its arena's bytes would take the resident volumes beyond volume_budget_bytes (the
 * server is unchanged); BUDGET or HIP if the first volume's workspaces cannot be laid out in
 * the arena.  The server may compound frames into it (dare_server_submit_frames); outside the
 * server the volume must not be reconstructed while the server can reslice it. */
dare_status dare_server_add_volume(dare_server* s, dare_volume* v, int32_t* volume_id);
/* Unregister a volume and return its bytes to the volume budget.  New requests for it are
 * refused (INVALID_ARG) from the call on; requests and frames jobs already queued still run.
 * The call waits up to wait_seconds for them to complete; if some are still pending then, it
 * returns NOT_READY and the volume stays registered.  INVALID_ARG for an unknown or removed id.
 * Ids are never reused; after OK the caller may destroy the volume. */
dare_status dare_server_remove_volume(dare_server* s, int32_t volume_id, double wait_seconds);
/* Device bytes and number of the volumes currently registered. */
dare_status dare_server_volume_bytes(dare_server* s, uint64_t* resident_bytes, int32_t* resident_volumes);
/* Queue a request.  host_out (required) receives height*width float32,
 * row-major, NaN where unassigned, once the request completes: host memory
 * (pinned or pageable) or device memory of the server's GPU, which must stay
 * valid until the ticket completes.  Returns
 * QUEUE_FULL when max_queue requests wait, and INVALID_ARG when the request
 * can never fit the arena's result space or one tick. */
dare_status dare_server_submit(dare_server* s, int32_t volume_id, const dare_slice_spec* spec,
                               float* host_out, uint64_t* ticket);
/* Queue a batch of tracked frames to compound into served volume `volume_id` (Sec. 2.1
 * "Volume reconstruction"; the streaming case: a probe keeps scanning while consoles reslice).
 * It takes its place in the request queue: requests submitted before it never see these
 * frames, requests submitted after it always do.  When it reaches the head of the queue the
 * scheduler lets the ticks in flight finish, compounds (dare_reconstruct_frames on one of the
 * server's streams) and resumes.  frames_dev (n*h*w uint8, row-major) and probe_poses_dev
 * (n*16 FP32, row-major) are device memory that must stay valid until the ticket completes;
 * pitch_mm is read before the call returns.  The ticket completes with the compounding status
 * (OK, WARN_BINS_SATURATED, BUDGET or BAD_POSE with the batch rolled back, HIP), which
 * dare_server_poll returns.  QUEUE_FULL as for dare_server_submit. */
dare_status dare_server_submit_frames(dare_server* s, int32_t volume_id, const uint8_t* frames_dev, int32_t n,
                                      int32_t w, int32_t h, const double pitch_mm[2], const float* probe_poses_dev,
                                      uint64_t* ticket);
/* Queue n requests in order under one lock (for gateways that receive
 * requests in groups).  Arrays of n: volume_ids, specs, host_outs (each
 * required); tickets receives one ticket per accepted request.  *accepted is
 * the number queued, a prefix of the n; the return value is DARE_OK when all
 * were, else the status of the first one refused (QUEUE_FULL, or INVALID_ARG
 * as for dare_server_submit), which and whose successors are not queued. */
dare_status dare_server_submit_many(dare_server* s, int32_t n, const int32_t* volume_ids,
                                    const dare_slice_spec* specs, float* const* host_outs,
                                    uint64_t* tickets, int32_t* accepted);
/* DARE_OK with *times filled (may be NULL) once the result is in its
 * host_out buffer, DARE_ERR_NOT_READY before, DARE_ERR_HIP if its tick failed; for a
 * frames ticket, its compounding status once compounded.  A ticket is
 * forgotten once poll has returned anything but NOT_READY. */
dare_status dare_server_poll(dare_server* s, uint64_t ticket, dare_request_times* times);
/* Poll n tickets at once: states[k] receives what dare_server_poll would
 * return for tickets[k] (times[k] filled when DARE_OK; times may be NULL),
 * and *n_done the number no longer NOT_READY (those tickets are forgotten).
 * With wait_seconds > 0 the call blocks, up to that long, until at least one
 * of the tickets has finished.  Returns INVALID_ARG only for bad arguments. */
dare_status dare_server_poll_many(dare_server* s, int32_t n, const uint64_t* tickets,
                                  dare_request_times* times, int32_t* states, double wait_seconds,
                                  int32_t* n_done);
/* Block until every submitted request has completed. */
dare_status dare_server_drain(dare_server* s);
dare_status dare_server_get_stats(dare_server* s, dare_server_stats* out);
/* Drain, stop the scheduler thread and release streams, graphs and staging (not the arena). */
dare_status dare_server_destroy(dare_server* s);
/* Steady-clock seconds used by the request times. */
double dare_now_seconds(void);

#ifdef __cplusplus
}
#endif

#endif /* DARE_H */
