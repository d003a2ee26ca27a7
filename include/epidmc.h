/*
 * epidmc.h -- C ABI of the MI355X (gfx950) EPID transit Monte Carlo engine.
 *
 * The engine transports photon histories and the electrons they set in motion
 * through a voxelised CT phantom and a multi-layer EPID, and tallies the energy
 * deposited in the EPID scoring layer into a 2D image with a per-pixel variance.
 * This is the patient and EPID part of the three-zone scheme of the paper
 * (Sec. 2.1, Fig. 1): particles leaving the treatment head (the second phase
 * space, Sec. 2.1.1) enter a density matrix derived from CT numbers (Sec. 2.1.2),
 * where photoelectric absorption, Compton scattering and pair production are
 * modelled for photons and a Class II condensed-history scheme for electrons,
 * with 10 keV and 200 keV cut-offs (Sec. 2.1.2); the particles crossing the exit
 * plane (the third phase space) continue into a stack of copper, reflector,
 * Gd2O2S and protective layers whose dose is scored on a pixel grid
 * (Sec. 2.1.3, Sec. 2.3.3).
 *
 * Units: cm, MeV, g/cm^3.  Coordinates: a right-handed frame whose z axis is the
 * beam axis; the EPID image is centred on x = y = 0, its u index runs along x and
 * its v index along y; images are row-major [v][u].
 *
 * Ownership and memory: the caller owns every host array passed in; set_* calls
 * validate and copy them into the context (host side) and return.  The engine
 * allocates no device memory: the caller queries epidmc_workspace_size() and
 * binds a device buffer of at least that size with epidmc_bind_workspace(),
 * which uploads the model.  Any set_* call after binding un-binds the context
 * (EPIDMC_E_NOT_READY) until the workspace is bound again.  Device pointers
 * (workspace, output images) are plain hipMalloc'd addresses, e.g. from PyTorch
 * tensors; streams are hipStream_t passed as void* (NULL = default stream).
 *
 * Errors: every call returns an epidmc_status; no exception crosses the ABI.
 * epidmc_last_error() returns a message for the last failed call on a context.
 * Device-side faults (queue overflow, step limit, sampler draw limit, NaN
 * energy, fixed-point overflow) are latched in a device error word and reported as
 * EPIDMC_E_OVERFLOW / EPIDMC_E_NAN by the next call that synchronises (run,
 * run_until, get_counters).  A context is not thread safe; use one per thread.
 */
#ifndef EPIDMC_H
#define EPIDMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct epidmc_ctx epidmc_ctx;

typedef enum {
    EPIDMC_OK = 0,
    EPIDMC_E_ARG = -1,        /* invalid argument value */
    EPIDMC_E_SHAPE = -2,      /* inconsistent sizes */
    EPIDMC_E_RANGE = -3,      /* value outside the supported range */
    EPIDMC_E_NOT_READY = -4,  /* model incomplete or workspace not bound */
    EPIDMC_E_WORKSPACE = -5,  /* workspace too small or misaligned */
    EPIDMC_E_DEVICE = -6,     /* HIP runtime error */
    EPIDMC_E_OVERFLOW = -7,   /* particle queue, step limit, sampler draw limit or fixed-point overflow */
    EPIDMC_E_NAN = -8         /* non-finite energy or position met on the device */
} epidmc_status;

typedef enum {
    EPIDMC_TALLY_FP64 = 0,     /* FP64 atomic adds into the image */
    EPIDMC_TALLY_FIXED64 = 1,  /* int64 fixed point, quantum 2^-32 MeV: bit-reproducible */
    EPIDMC_TALLY_KAHAN32 = 2   /* deposit records reduced per tile with Kahan-compensated FP32 */
} epidmc_tally_mode;

typedef enum {
    EPIDMC_PHYS_KERMA = 0,    /* electrons deposit their kinetic energy where they are set in motion */
    EPIDMC_PHYS_COUPLED = 1   /* electrons are transported by condensed history */
} epidmc_phys_mode;

/* process mask bits */
#define EPIDMC_PROC_COMPTON  1u
#define EPIDMC_PROC_PHOTO    2u
#define EPIDMC_PROC_PAIR     4u
#define EPIDMC_DIAG_NO_HARD  8u    /* diagnostic: no discrete electron events */
#define EPIDMC_DIAG_NO_MSC  16u    /* diagnostic: no multiple scattering */

#define EPIDMC_MAX_ELEM 8
#define EPIDMC_MAX_MATERIALS 16
#define EPIDMC_MAX_PHANTOM_MATERIALS 4   /* materials present in one phantom */
#define EPIDMC_MAX_LAYERS 6
#define EPIDMC_MAX_SEGMENTS 256
#define EPIDMC_MAX_BATCH_SLOTS 128

/* A material: elemental composition by mass fraction and mean excitation energy. */
typedef struct {
    int    n_elem;
    int    Z[EPIDMC_MAX_ELEM];
    double A[EPIDMC_MAX_ELEM];   /* g/mol */
    double w[EPIDMC_MAX_ELEM];   /* mass fractions (normalised by the engine) */
    double I_eV;                 /* mean excitation energy */
} epidmc_material;

/* CT number -> density (piecewise linear over n_points ascending HU, clamped outside)
 * and CT number -> material (material[r] for HU < hu_upper[r], first match; the last
 * range, r = n_ranges-1, takes everything else and its hu_upper is ignored).  This is the
 * HU-to-density conversion of Sec. 2.1.2, with the curve supplied by the caller. */
typedef struct {
    int           n_points;
    const double *hu;
    const double *rho;
    int           n_ranges;
    const double *hu_upper;
    const int    *material;
} epidmc_hu_curve;

/* One EPID layer: material index, thickness along z (cm), density (g/cm^3). */
typedef struct {
    int   material;
    float thickness;
    float density;
} epidmc_layer;

/* Beam: kind 0 = parallel beam along +z starting on the plane z = src[2], with the
 * aperture defining (x, y) on that plane; kind 1 = point source at src aimed at a
 * point drawn uniformly over the open aperture area on the plane z = iso_z. */
typedef struct {
    int   kind;
    float src[3];
    float iso_z;
} epidmc_beam;

/* A phase-space particle (global frame): type 0 photon, 1 electron. */
typedef struct {
    float x, y, z, u, v, w, E;
    int   type;
} epidmc_particle;

typedef struct {
    uint64_t histories;            /* histories transported since the last reset */
    uint64_t n_compton, n_photo, n_pair, n_annih, n_brems, n_moller;
    uint64_t woodcock_steps;       /* real + virtual delta-tracking steps in the phantom */
    uint64_t epid_photon_steps;    /* photon flights in the EPID slabs */
    uint64_t e_steps_phantom, e_steps_epid;
    uint64_t photon_epid_entries, unscattered_at_epid;
    uint64_t tally_deposits;
    uint64_t queue_items[4];       /* particles consumed per queue: photon-phantom,
                                      electron-phantom, photon-EPID, electron-EPID */
    uint64_t lane_iters[4];        /* per queue kernel: sum over wave iterations of active lanes */
    uint64_t wave_iters[4];        /* per queue kernel: wave iterations x 64 */
    uint64_t launches;             /* transport kernel launches */
    uint64_t queue_peak;           /* largest queue fill seen */
    uint32_t error_word;           /* latched device error bits */
    double   max_ledger_resid;     /* diagnostics on: max per-history |E_in - deposited - escaped
                                      - net rest energy| / E_in */
    double   e_in, e_deposited, e_escaped;
    double   kernel_ms[4];         /* profiling on: summed HIP-event durations of the transport
                                      kernels per queue kind (same order as queue_items) */
    uint64_t kernel_launches[4];
} epidmc_counters;

/* ---- lifetime ---------------------------------------------------------------- */
/* Create a context on HIP device `device`; `seed` keys the counter-based random
 * streams (Philox4x32-10, one stream per history and particle). */
epidmc_status epidmc_create(epidmc_ctx **out, int device, uint64_t seed);
epidmc_status epidmc_destroy(epidmc_ctx *c);
/* Message of the last failed call; valid until the next call on c. */
const char *epidmc_last_error(const epidmc_ctx *c);

/* ---- model ------------------------------------------------------------------- */
/* Material table; phantom and EPID layers refer to materials by index. */
epidmc_status epidmc_set_materials(epidmc_ctx *c, const epidmc_material *m, int n_materials);
/* Physics: transport mode, process mask (EPIDMC_PROC_* | EPIDMC_DIAG_*), cut-offs in
 * MeV (the paper's 0.010 photon and 0.200 electron cut-offs, Sec. 2.1.2).  Kinetic
 * energies below a cut-off are deposited on the spot. */
epidmc_status epidmc_set_physics(epidmc_ctx *c, epidmc_phys_mode mode, uint32_t process_mask,
                                 float photon_cut_MeV, float electron_cut_MeV);
/* Phantom from CT numbers, x fastest: hu[(k*ny + j)*nx + i]; spacing and origin (the
 * minimum corner) in cm.  The curve maps HU to (material, density) (Sec. 2.1.2). */
epidmc_status epidmc_set_phantom_hu(epidmc_ctx *c, const int16_t *hu, int nx, int ny, int nz,
                                    const float spacing[3], const float origin[3],
                                    const epidmc_hu_curve *curve);
/* Phantom from per-voxel material index and density. */
epidmc_status epidmc_set_phantom_direct(epidmc_ctx *c, const uint8_t *mat, const float *rho,
                                        int nx, int ny, int nz, const float spacing[3],
                                        const float origin[3]);
/* EPID: contiguous layers from z = front_z downstream (Sec. 2.1.3), the index of the
 * scoring layer, and the image: npx_u x npx_v pixels of pitch_u x pitch_v centred on
 * the axis (Sec. 2.3.3).  The lateral extent of every layer is the image area. */
epidmc_status epidmc_set_epid(epidmc_ctx *c, const epidmc_layer *layers, int n_layers, int scoring_layer,
                              float front_z, int npx_u, int npx_v, float pitch_u, float pitch_v);
/* Source spectrum: nbins bins with edges[nbins+1] (non-decreasing, MeV) and
 * non-negative weights[nbins]; energy uniform within the chosen bin (a zero-width bin is
 * a line).  Replaces any phase-space list. */
epidmc_status epidmc_set_source_spectrum(epidmc_ctx *c, const float *edges_MeV, const float *weights,
                                         int nbins, const epidmc_beam *beam);
/* Phase-space list (the particles after the collimators, Sec. 2.1.1): history h
 * starts from particle h mod n.  Replaces the spectrum and aperture sampling. */
epidmc_status epidmc_set_source_phsp(epidmc_ctx *c, const epidmc_particle *p, uint64_t n);
/* MLC apertures on the beam's aperture plane: leaf pair k of segment s spans y in
 * [y0 + k*w, y0 + (k+1)*w) and is open for x in [a[s*n_pairs+k], b[s*n_pairs+k]]
 * (the apertures of Sec. 2.1.1, taken from the plan).  Global history ids are assigned
 * to segments consecutively by n_hist[s] (ids past their total repeat the delivery, see
 * epidmc_run); with one segment n_hist is ignored. */
epidmc_status epidmc_set_segments(epidmc_ctx *c, int n_segments, int n_pairs, float leaf_width, float y0,
                                  const float *a, const float *b, const uint64_t *n_hist);
/* Tally: mode, variance batches per run call (>= 2; 64 or more recommended), and the
 * largest number of histories processed together (sets queue capacities). */
epidmc_status epidmc_set_tally(epidmc_ctx *c, epidmc_tally_mode mode, int batches_per_run,
                               uint64_t max_chunk_histories);
/* Diagnostics: when on, every history's energy ledger is kept on the device and checked. */
epidmc_status epidmc_set_diagnostics(epidmc_ctx *c, int enable);
/* Profiling: when on, every transport launch is bracketed by HIP events on the stream it
 * runs on and the durations are summed into epidmc_counters.kernel_ms. */
epidmc_status epidmc_set_profiling(epidmc_ctx *c, int enable);

/* Queue passes (the regrouping of Sec. 2.1's transport into per-kind work queues): the first
 * `device_passes` passes of each chunk of histories are launched without waiting for the host
 * (every particle kind at its resident grid size, blocks beyond the queue's need leaving at
 * once on the device); the host reads the queues back once after them and drives any further
 * passes itself.  -1 (the default): as many device-driven passes as the previous chunk had
 * non-empty ones; 0: host-driven throughout.  Grids are sized for about `items_per_lane`
 * queued particles per lane (default 2).  Neither changes any trajectory: a fixed-point image
 * is the same bit for bit for every setting.  EPIDMC_E_ARG outside [-1, 24] and [1, 64]. */
epidmc_status epidmc_set_passes(epidmc_ctx *c, int device_passes, int items_per_lane);
/* Graph runs (the batched delivery of a whole IMRT field, Sec. 2.3: all segments of a run in
 * one launch): when enabled, a run call for a history range captures the whole run -- every
 * chunk's source and `passes` device-driven queue passes (0: the previous chunk's non-empty
 * passes plus two, or 12 before any chunk ran), and the folds -- as one HIP graph on a stream
 * of the library's own, and replays it on `stream`; a later call with the same history range
 * replays the graph (the same histories again: the tally adds them once more).  A run whose
 * queues still hold particles after the captured passes returns EPIDMC_E_OVERFLOW (its tally
 * is then incomplete: reset it and raise `passes`).  Needs the FP64 or fixed-point tally and
 * diagnostics off (EPIDMC_E_ARG otherwise); profiling events are not recorded in graph runs.
 * Any set_* call or a new workspace drops the captured graph. */
epidmc_status epidmc_set_graph(epidmc_ctx *c, int enable, int passes);

/* ---- memory ------------------------------------------------------------------ */
epidmc_status epidmc_workspace_size(epidmc_ctx *c, size_t *bytes);
/* Bind caller-owned device memory (256-byte aligned, >= workspace_size bytes) and
 * upload the model on `stream`.  Clears the tally. */
epidmc_status epidmc_bind_workspace(epidmc_ctx *c, void *dev_ptr, size_t bytes, void *stream);

/* ---- run --------------------------------------------------------------------- */
/* Transport histories [first_history, first_history + n_histories) on `stream`, split
 * into the configured number of variance batches, and fold them into the tally.
 * Returns after the work has completed.  History ids are 64-bit: the random stream of
 * history h is keyed by the seed and h's high 32 bits, and counted by its low 32 bits, so
 * ids below 2^32 keep the plain seed key.  A segmented field of total T histories takes
 * ids [0, T) as one delivery; an id h >= T belongs to delivery h / T and samples the
 * segment of h mod T with its own random stream, so consecutive id ranges deliver the field
 * again with independent histories.
 * Within a queue pass the four particle kinds run concurrently: three on streams the
 * context creates (default priority) and the last on `stream`, which waits for the
 * others before the next pass. */
epidmc_status epidmc_run(epidmc_ctx *c, uint64_t first_history, uint64_t n_histories, void *stream);
/* Run chunks of `step_histories` from history `first_history` until the mean relative
 * standard deviation over pixels with D >= threshold_frac * max(D) is <= target, or
 * max_histories have been run.  Reports histories run and the last sigma-bar. */
epidmc_status epidmc_run_until(epidmc_ctx *c, double target_rel_unc, double threshold_frac,
                               uint64_t first_history, uint64_t step_histories, uint64_t max_histories,
                               void *stream, uint64_t *histories_done, double *sigma_bar);
/* Mean energy per history (MeV) and the variance of that mean (MeV^2), [npx_v][npx_u]
 * FP64, written to caller device buffers on `stream` (asynchronous). */
epidmc_status epidmc_read_image(epidmc_ctx *c, double *dev_mean, double *dev_var, void *stream);
/* Mean relative standard deviation over pixels with D >= threshold_frac * max(D). */
epidmc_status epidmc_sigma_bar(epidmc_ctx *c, double threshold_frac, void *stream, double *out);
epidmc_status epidmc_reset_tally(epidmc_ctx *c, void *stream);
/* Work and diagnostic counters accumulated since the last reset (synchronises). */
epidmc_status epidmc_get_counters(epidmc_ctx *c, epidmc_counters *out);

/* ---- dose-response correction (Sec. 2.2, Sec. 3.1) ---------------------------- */
/* Radiological thickness map (Sec. 2.2, item 1): for every pixel, the line integral of the
 * phantom's density divided by 1 g/cm^3 (cm) along the ray from the point source to the
 * pixel centre on the mid-plane of the scoring layer, or along +z through the pixel centre
 * for a parallel beam.  dev_out: device pointer to npx_u * npx_v doubles, row-major with u
 * fastest (the image layout).  Needs a bound workspace, whose packed phantom it reads
 * (densities within 2^-21 relative).  Runs on `stream` and returns without waiting.
 * EPIDMC_E_NOT_READY if unbound, EPIDMC_E_ARG for a null pointer. */
epidmc_status epidmc_radiological_thickness(epidmc_ctx *c, double *dev_out, void *stream);
/* Effective field size (Sec. 2.2, item 2; Eq. 1 read as 4A/P), in cm: the equivalent
 * square 2ab/(a+b) of the a x b bounding rectangle of the open leaf pairs (b > a) of all
 * segments, on the aperture plane.  Host computation, no device work.  EPIDMC_E_NOT_READY
 * without an aperture (a phase-space source) or with every leaf pair closed. */
epidmc_status epidmc_field_size(epidmc_ctx *c, double *s_out);
/* Dose-response correction (Sec. 3.1, Eq. 2 and Table 1): dev_out[p] = k(dev_t[p], s) *
 * dev_image[p] for the npx_u * npx_v pixels.  k is bilinear on the rectilinear table
 * t_nodes[nt], s_nodes[ns] (strictly ascending), k[j*nt + i] the factor at (t_i, s_j),
 * 1 <= nt, ns <= 64, in host memory; outside the table t and s are clamped to its edges.
 * dev_image, dev_t and dev_out are device pointers to doubles (dev_out may equal
 * dev_image).  Runs on `stream` and returns without waiting.  EPIDMC_E_ARG / E_RANGE for
 * bad pointers, sizes, unordered nodes or non-finite values. */
epidmc_status epidmc_dose_response(epidmc_ctx *c, const double *dev_image, const double *dev_t, double s,
                                   const double *t_nodes, int nt, const double *s_nodes, int ns,
                                   const double *k, double *dev_out, void *stream);

/* Resample a k(t,s) table onto other nodes (Sec. 3.1: Table 1 resampled onto the finer
 * 64 x 64 table of a large field, up to 64 nodes per axis): k_out[j*mt + i] = k(t_out[i],
 * s_out[j]), with k bilinear on t_nodes[nt] x s_nodes[ns] (k[j*nt + i] at (t_i, s_j)) and t, s
 * clamped to the table's edges, exactly as epidmc_dose_response evaluates it.  When the new
 * nodes include the old ones, the new table interpolates to the same function.  Host
 * arrays; host computation, no device work.  EPIDMC_E_ARG for null pointers, EPIDMC_E_RANGE
 * for sizes outside 1..64, unordered nodes or non-finite values. */
epidmc_status epidmc_resample_response_table(const double *t_nodes, int nt, const double *s_nodes, int ns,
                                             const double *k, const double *t_out, int mt, const double *s_out,
                                             int ms, double *k_out);

/* ---- diagnostics of the device building blocks (test entry points) ----------- */
/* Philox4x32-10 on the device: out[4*i..4*i+3] = philox(ctr[4*i..], key).  Device pointers. */
epidmc_status epidmc_debug_philox(epidmc_ctx *c, const uint32_t *dev_ctr, uint32_t *dev_out, uint64_t n,
                                  void *stream);
/* Device samplers: kind 0 Klein-Nishina eps = E'/E at energy p0; kind 1 Moller energy
 * transfer at kinetic energy p0; kind 2 bremsstrahlung photon energy at p0; kind 3
 * multiple-scattering polar angle for kinetic energy p0 over p1 g/cm^2 of material p2;
 * kind 4 the source: 8 floats (x y z u v w E type) per history for histories
 * [p0, p0 + n), p0 an integer below 2^53 and the range within one 2^32 block, drawn by the
 * source kernel's own sampling function with its key; kind 5 the azimuth uniform that
 * accompanies a kind-0 sample (uniform on (0, 1)).  n samples into dev_out. */
epidmc_status epidmc_debug_sample(epidmc_ctx *c, int kind, double p0, double p1, double p2, float *dev_out,
                                  uint64_t n, void *stream);
/* Test entry point for the queue-overflow path: the capacity of every segment of queue
 * `kind` (1 electrons in the phantom, 2 photons in the EPID, 3 electrons in the EPID; the
 * phantom photon queue, which the source fills by slot, cannot be changed) in particles, from
 * the next epidmc_bind_workspace on (the call unbinds); 0 restores the capacity derived from
 * max_chunk_histories, at most 2^24.  A pass whose appends exceed a segment stores nothing
 * beyond it, drops the particles that do not fit and latches the overflow, which the run
 * returns as EPIDMC_E_OVERFLOW; the image of such a run is incomplete until the next bind. */
epidmc_status epidmc_debug_queue_capacity(epidmc_ctx *c, int kind, uint32_t per_segment);
/* Deposit records of the last chunk transported in the Kahan tally mode, the tally's raw
 * input (a test entry point: re-binned on the host they must give the tally): up to cap
 * records copied on `stream` to dev_pix (image element = variance-batch slot * npx_u * npx_v
 * + pixel index) and dev_e (MeV, FP32); *n receives the chunk's record count, which may
 * exceed cap.  Device pointers.  EPIDMC_E_NOT_READY outside the Kahan mode or before a run. */
epidmc_status epidmc_debug_records(epidmc_ctx *c, uint32_t *dev_pix, float *dev_e, uint64_t cap, uint64_t *n,
                                   void *stream);
/* The device cross-section tables evaluated at energies: kind 0 photon mu/rho of
 * material slot `index` (phantom slots 0..3, EPID layers 4..), kind 1 electron range,
 * kind 2 electron hard cross section (phantom slots 0..3, EPID layers 4..). */
epidmc_status epidmc_debug_table(epidmc_ctx *c, int kind, int index, const float *dev_E, float *dev_out,
                                 uint64_t n, void *stream);

/* ---- measurement probes (no part of the transport) ----------------------------- */
/* Kernels that measure the peaks the transport kernels' rates are compared with, on the GPU
 * that runs them.  dev_buf: caller-owned device memory of `bytes` bytes, contents
 * overwritten.  kind 0: streaming copy of the first half of dev_buf into the second half
 * (16-byte words; the other arguments are ignored).  kind 1: `threads` threads (a multiple of
 * 256) each make ops_per_thread 4-byte loads at pseudo-random indices of a table of
 * 2^log2_elems words at the start of dev_buf.  kind 2 / 3: the same pattern of FP64 / int64
 * atomic adds (no returned value) into a table of 2^log2_elems 8-byte words, log2_elems 6
 * concentrating them on 64 hot words.  Asynchronous on `stream`; the caller times it.
 * EPIDMC_E_ARG for a bad kind, thread count or log2_elems outside 1..31; EPIDMC_E_WORKSPACE
 * when the table does not fit in `bytes`. */
epidmc_status epidmc_microbench(int kind, void *dev_buf, size_t bytes, int log2_elems, uint32_t ops_per_thread,
                                uint32_t threads, void *stream);

#ifdef __cplusplus
}
#endif
#endif
