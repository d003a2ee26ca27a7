// epidmc.cpp -- C ABI, model validation, workspace layout and the queue-pass orchestrator.
#include "../../include/epidmc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"
#include "tables.hpp"

namespace epidmc {
hipError_t launch_source(const Params &P, hipStream_t s);
hipError_t launch_transport(int kind, const Params &P, unsigned blocks, hipStream_t s);
size_t lds_bytes(int kind, const Params &P);
hipError_t set_lds_limits();
hipError_t launch_fold(const Params &P, const int *slots, const double *nb, int n, hipStream_t s);
hipError_t launch_kahan_reduce(const Params &P, uint32_t nrec, uint32_t nimg, uint32_t *count, uint32_t *cursor,
                               uint32_t *bsum, float *sorted, hipStream_t s);
hipError_t launch_image(const Params &P, double n, double nb, double *mean, double *var, hipStream_t s);
hipError_t launch_sigma_bar(const Params &P, double n, double nb, double thr, double *out, hipStream_t s);
hipError_t launch_diag_check(const Params &P, uint32_t nh, unsigned long long *maxbits, double *sums, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_pass_start(const Params &P, const uint32_t *cnt, uint32_t *tot, uint32_t *fills, uint32_t *heads,
                             size_t words, hipStream_t s, uint32_t *hist);
hipError_t launch_radthick(const RadArgs &A, hipStream_t s);
hipError_t launch_response(const RespArgs &A, hipStream_t s);
hipError_t launch_dbg_philox(const Params &P, const uint32_t *ctr, uint32_t *out, unsigned long long n, hipStream_t s);
hipError_t launch_dbg_sample(const Params &P, int kind, float p0, float p1, float p2, float *out,
                             unsigned long long n, hipStream_t s);
hipError_t launch_dbg_table(const Params &P, int kind, int index, const float *E, float *out, unsigned long long n,
                            hipStream_t s);
hipError_t launch_dbg_source(const Params &P, unsigned long long h0, float *out, unsigned long long n, hipStream_t s);
}  // namespace epidmc

using namespace epidmc;

namespace {

struct Region {
    size_t off, bytes;
};

struct Layout {
    Region vox, ph_tab, ph_maj, ph_mu4, ph_fr, el_tab, sp_lo, sp_hi, sp_prob, sp_alias, ap_a, ap_b, ap_prob, ap_alias, seg_end,
        phsp, ctl, segc, queues, img, sum, sum2, led, ein, rec_pix, rec_e, k_count, k_cursor, k_bsum, k_sorted;
    size_t total;
    uint32_t cap[NQ];          // particles per queue: NSEG segments of segcap
    uint32_t segcap[NQ];
    uint32_t rec_cap;
    int ring;
    uint64_t chunk;
};

constexpr size_t CTL_CNT = 0;                 // 16 u32: [NQ] particles per queue after a pass, [3 NQ] record count
constexpr size_t SEG_SET = (size_t)NQ * NSEG * CSTRIDE;   // u32 words of one set of segment counters
constexpr size_t CTL_ERR = 64;                // u32
constexpr size_t CTL_STATS = 128;             // S_NSTAT u64
constexpr size_t CTL_DIAG = CTL_STATS + 8 * 32;   // max-residual bits, e_in, e_ledger
constexpr size_t CTL_SIGMA = CTL_DIAG + 64;   // double
constexpr int MAX_DEV_PASSES = 24;            // device-driven passes per chunk (at most)
constexpr int MAX_GRAPH_CHUNKS = 32;          // chunks of one captured run (at most)
constexpr size_t CTL_PASSHIST = 512;          // [MAX_DEV_PASSES][NQ + 1] u32: per-pass totals and error word
constexpr size_t CTL_LEFT = 1024;             // [MAX_GRAPH_CHUNKS][NQ + 1] u32: totals after a captured chunk's last pass
constexpr size_t CTL_BYTES = CTL_LEFT + (size_t)MAX_GRAPH_CHUNKS * (NQ + 1) * 4;

}  // namespace

struct epidmc_ctx {
    int device = 0;
    uint64_t seed = 0;
    std::string err;
    int n_cu = 256;
    // model
    std::vector<HostMaterial> mats;
    int coupled = 1;
    uint32_t mask = 7u;
    float pcut = 0.010f, ecut = 0.200f;
    int nx = 0, ny = 0, nz = 0;
    float spacing[3] = {0, 0, 0}, origin[3] = {0, 0, 0};
    std::vector<uint8_t> vmat;     // global material index per voxel
    std::vector<float> vrho;
    std::vector<epidmc_layer> layers;
    int scoring = 0;
    float front_z = 0;
    int npx_u = 0, npx_v = 0;
    float pitch_u = 0, pitch_v = 0;
    std::vector<float> edges, weights;
    epidmc_beam beam{};
    bool have_spectrum = false;
    std::vector<float> phsp;
    uint64_t n_phsp = 0;
    int n_seg = 0, n_pairs = 0;
    float leaf_w = 0, y0 = 0;
    std::vector<float> ap_a, ap_b;
    std::vector<uint64_t> seg_hist;
    int tally_mode = 0, batches = 64;
    uint64_t max_chunk = 1ull << 21;
    int diag = 0;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    Layout lay{};
    Params P{};
    Queue qs[2][NQ];                // the two queue buffer sets
    int slot_of_mat[EPIDMC_MAX_MATERIALS];
    uint32_t *host = nullptr;       // pinned readback area
    int occ[NQ] = {1, 1, 1, 1};
    // profiling
    int prof = 0;
    hipEvent_t ev[2][NQ] = {};
    // the kinds of a pass run concurrently, so a pass lasts as long as its slowest kernel
    // rather than the sum of them: kinds 0..NQ-2 on streams of their own, the last kind on
    // the run stream itself, so that the run takes NQ streams, as many as the hardware
    // queues a process gets by default (a fifth stream would share a queue with another
    // and serialise behind it)
    hipStream_t ks[NQ] = {};
    hipEvent_t go = nullptr, done[NQ] = {};
    double kernel_ms[NQ] = {0, 0, 0, 0};
    uint64_t kernel_launches[NQ] = {0, 0, 0, 0};
    uint32_t last_nrec = 0;         // Kahan mode: records of the last chunk
    // passes: the first `dev_passes` passes of a chunk are launched without a host round trip
    // (-1: as many as the previous chunk had non-empty passes); grids for about `ipl` items
    // per lane
    int dev_passes = -1, last_passes = 0, ipl = ITEMS_PER_LANE;
    hipEvent_t dev_ev[MAX_DEV_PASSES][2][NQ] = {};
    // the previous chunk's queue totals per pass (zero where a queue was empty or the pass did
    // not run), from which device-driven passes size their grids
    uint32_t prev_rows[MAX_DEV_PASSES][NQ] = {};
    bool have_rows = false;
    // a whole run captured as one graph (FP64 or fixed-point tally, diagnostics off), replayed
    // while the run's history range is the same
    int graph = 0, graph_passes = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t gx = nullptr;
    uint64_t g_first = 0, g_n = 0;
    int g_chunks = 0, g_passes = 0;
    hipStream_t cap = nullptr;      // the stream a run is captured on (capture needs a stream other than the null stream)
    uint64_t graph_launches = 0;
    // accumulated
    double n_total = 0, b_total = 0;
    uint64_t launches = 0, queue_peak = 0;
    uint32_t q_override[NQ] = {0, 0, 0, 0};   // test hook: particles per segment (0: derived)
};

static epidmc_status fail(epidmc_ctx *c, epidmc_status s, const std::string &m)
{
    if (c) c->err = m;
    return s;
}
#define REQUIRE(cond, code, msg) \
    do { if (!(cond)) return fail(c, code, msg); } while (0)
#define HIPCHK(x)                                                                                          \
    do {                                                                                                   \
        hipError_t e_ = (x);                                                                               \
        if (e_ != hipSuccess) return fail(c, EPIDMC_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool finite3(const float v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

static void drop_graph(epidmc_ctx *c);

// a change of the model invalidates the workspace and any captured run
static void unbind(epidmc_ctx *c)
{
    c->bound = false;
    drop_graph(c);
}

extern "C" {

epidmc_status epidmc_create(epidmc_ctx **out, int device, uint64_t seed)
{
    if (!out) return EPIDMC_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EPIDMC_E_DEVICE;
    epidmc_ctx *c = new epidmc_ctx();
    c->device = device;
    c->seed = seed;
    if (hipSetDevice(device) != hipSuccess) { delete c; return EPIDMC_E_DEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    if (hipHostMalloc((void **)&c->host, 4096, hipHostMallocDefault) != hipSuccess) { delete c; return EPIDMC_E_DEVICE; }
    // raise the dynamic LDS cap of the transport kernels where the device allows it; the
    // default cap already covers up to five EPID layers
    (void)set_lds_limits();
    (void)hipGetLastError();
    *out = c;
    return EPIDMC_OK;
}

epidmc_status epidmc_destroy(epidmc_ctx *c)
{
    if (!c) return EPIDMC_E_ARG;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < NQ; ++k)
            if (c->ev[b][k]) (void)hipEventDestroy(c->ev[b][k]);
    for (int k = 0; k < NQ; ++k) {
        if (c->done[k]) (void)hipEventDestroy(c->done[k]);
        if (c->ks[k]) (void)hipStreamDestroy(c->ks[k]);
    }
    if (c->go) (void)hipEventDestroy(c->go);
    for (int p = 0; p < MAX_DEV_PASSES; ++p)
        for (int b = 0; b < 2; ++b)
            for (int k = 0; k < NQ; ++k)
                if (c->dev_ev[p][b][k]) (void)hipEventDestroy(c->dev_ev[p][b][k]);
    if (c->gx) (void)hipGraphExecDestroy(c->gx);
    if (c->g) (void)hipGraphDestroy(c->g);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
    return EPIDMC_OK;
}

const char *epidmc_last_error(const epidmc_ctx *c) { return c ? c->err.c_str() : "null context"; }

epidmc_status epidmc_set_materials(epidmc_ctx *c, const epidmc_material *m, int n)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(m && n >= 1 && n <= EPIDMC_MAX_MATERIALS, EPIDMC_E_ARG, "1..16 materials required");
    std::vector<HostMaterial> v(n);
    for (int i = 0; i < n; ++i) {
        REQUIRE(m[i].n_elem >= 1 && m[i].n_elem <= EPIDMC_MAX_ELEM, EPIDMC_E_ARG, "material element count");
        REQUIRE(std::isfinite(m[i].I_eV) && m[i].I_eV > 0, EPIDMC_E_ARG, "material I-value must be > 0");
        double ws = 0;
        v[i].n = m[i].n_elem;
        for (int k = 0; k < m[i].n_elem; ++k) {
            REQUIRE(m[i].Z[k] >= 1 && m[i].Z[k] <= 100, EPIDMC_E_RANGE, "element Z out of range");
            REQUIRE(std::isfinite(m[i].A[k]) && m[i].A[k] > 0, EPIDMC_E_ARG, "element A must be > 0");
            REQUIRE(std::isfinite(m[i].w[k]) && m[i].w[k] >= 0, EPIDMC_E_ARG, "mass fraction must be >= 0");
            v[i].Z[k] = m[i].Z[k];
            v[i].A[k] = m[i].A[k];
            v[i].w[k] = m[i].w[k];
            ws += m[i].w[k];
        }
        REQUIRE(ws > 0, EPIDMC_E_ARG, "mass fractions sum to zero");
        v[i].I_eV = m[i].I_eV;
    }
    c->mats = v;
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_physics(epidmc_ctx *c, epidmc_phys_mode mode, uint32_t mask, float pcut, float ecut)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(mode == EPIDMC_PHYS_KERMA || mode == EPIDMC_PHYS_COUPLED, EPIDMC_E_ARG, "unknown physics mode");
    REQUIRE((mask & 7u) != 0 && mask < 32u, EPIDMC_E_ARG, "process mask needs a photon process, bits 0..4 only");
    REQUIRE(std::isfinite(pcut) && pcut >= 1e-3f && pcut < 1.0f, EPIDMC_E_RANGE, "photon cut-off in [1 keV, 1 MeV)");
    REQUIRE(std::isfinite(ecut) && ecut >= 0.05f && ecut < 2.0f, EPIDMC_E_RANGE, "electron cut-off in [50 keV, 2 MeV)");
    REQUIRE(ecut >= (float)WCUT - 1e-6f || mode == EPIDMC_PHYS_KERMA, EPIDMC_E_RANGE,
            "coupled transport needs an electron cut-off >= the 200 keV Moller threshold");
    c->coupled = mode == EPIDMC_PHYS_COUPLED;
    c->mask = mask;
    c->pcut = pcut;
    c->ecut = ecut;
    unbind(c);
    return EPIDMC_OK;
}

static epidmc_status check_grid(epidmc_ctx *c, int nx, int ny, int nz, const float sp[3], const float org[3])
{
    REQUIRE(nx > 0 && ny > 0 && nz > 0, EPIDMC_E_SHAPE, "phantom dimensions must be > 0");
    REQUIRE((uint64_t)nx * ny * nz <= (1ull << 31), EPIDMC_E_RANGE, "phantom larger than 2^31 voxels");
    REQUIRE(sp && org && finite3(sp) && finite3(org), EPIDMC_E_ARG, "spacing/origin must be finite");
    REQUIRE(sp[0] > 0 && sp[1] > 0 && sp[2] > 0, EPIDMC_E_ARG, "spacing must be > 0");
    return EPIDMC_OK;
}

epidmc_status epidmc_set_phantom_direct(epidmc_ctx *c, const uint8_t *mat, const float *rho, int nx, int ny, int nz,
                                        const float sp[3], const float org[3])
{
    if (!c) return EPIDMC_E_ARG;
    epidmc_status s = check_grid(c, nx, ny, nz, sp, org);
    if (s != EPIDMC_OK) return s;
    REQUIRE(mat && rho, EPIDMC_E_ARG, "null phantom arrays");
    const size_t n = (size_t)nx * ny * nz;
    for (size_t i = 0; i < n; ++i) {
        REQUIRE(std::isfinite(rho[i]) && rho[i] >= 0.0f && rho[i] < 1e4f, EPIDMC_E_ARG, "voxel density must be finite and >= 0");
        REQUIRE(mat[i] < c->mats.size(), EPIDMC_E_RANGE, "voxel material index not in the material table");
    }
    c->vmat.assign(mat, mat + n);
    c->vrho.assign(rho, rho + n);
    c->nx = nx; c->ny = ny; c->nz = nz;
    std::memcpy(c->spacing, sp, sizeof c->spacing);
    std::memcpy(c->origin, org, sizeof c->origin);
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_phantom_hu(epidmc_ctx *c, const int16_t *hu, int nx, int ny, int nz, const float sp[3],
                                    const float org[3], const epidmc_hu_curve *cv)
{
    if (!c) return EPIDMC_E_ARG;
    epidmc_status s = check_grid(c, nx, ny, nz, sp, org);
    if (s != EPIDMC_OK) return s;
    REQUIRE(hu && cv && cv->hu && cv->rho && cv->hu_upper && cv->material, EPIDMC_E_ARG, "null HU inputs");
    REQUIRE(cv->n_points >= 1 && cv->n_ranges >= 1, EPIDMC_E_ARG, "HU curve needs points and ranges");
    for (int k = 0; k < cv->n_points; ++k) {
        REQUIRE(std::isfinite(cv->hu[k]) && std::isfinite(cv->rho[k]) && cv->rho[k] >= 0, EPIDMC_E_ARG, "HU curve values");
        if (k) REQUIRE(cv->hu[k] > cv->hu[k - 1], EPIDMC_E_ARG, "HU curve points must ascend");
    }
    for (int r = 0; r < cv->n_ranges; ++r)
        REQUIRE(cv->material[r] >= 0 && cv->material[r] < (int)c->mats.size(), EPIDMC_E_RANGE,
                "HU range material not in the material table");
    const size_t n = (size_t)nx * ny * nz;
    std::vector<uint8_t> m(n);
    std::vector<float> rho(n);
    for (size_t i = 0; i < n; ++i) {
        const double x = hu[i];
        double r;
        if (x <= cv->hu[0]) r = cv->rho[0];
        else if (x >= cv->hu[cv->n_points - 1]) r = cv->rho[cv->n_points - 1];
        else {
            int k = 0;
            while (!(x < cv->hu[k + 1])) ++k;
            r = cv->rho[k] + (cv->rho[k + 1] - cv->rho[k]) * (x - cv->hu[k]) / (cv->hu[k + 1] - cv->hu[k]);
        }
        int rr = cv->n_ranges - 1;
        for (int k = 0; k < cv->n_ranges - 1; ++k)
            if (x < cv->hu_upper[k]) { rr = k; break; }
        m[i] = (uint8_t)cv->material[rr];
        rho[i] = (float)r;
    }
    c->vmat.swap(m);
    c->vrho.swap(rho);
    c->nx = nx; c->ny = ny; c->nz = nz;
    std::memcpy(c->spacing, sp, sizeof c->spacing);
    std::memcpy(c->origin, org, sizeof c->origin);
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_epid(epidmc_ctx *c, const epidmc_layer *layers, int nl, int scoring, float front_z, int npx_u,
                              int npx_v, float pitch_u, float pitch_v)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(layers && nl >= 1 && nl <= EPIDMC_MAX_LAYERS, EPIDMC_E_ARG, "1..6 EPID layers");
    REQUIRE(scoring >= 0 && scoring < nl, EPIDMC_E_RANGE, "scoring layer index");
    REQUIRE(std::isfinite(front_z), EPIDMC_E_ARG, "front_z must be finite");
    REQUIRE(npx_u > 0 && npx_v > 0 && (uint64_t)npx_u * npx_v <= (1ull << 26), EPIDMC_E_SHAPE, "image size");
    REQUIRE(std::isfinite(pitch_u) && std::isfinite(pitch_v) && pitch_u > 0 && pitch_v > 0, EPIDMC_E_ARG, "pitch must be > 0");
    for (int l = 0; l < nl; ++l) {
        REQUIRE(layers[l].material >= 0 && layers[l].material < (int)c->mats.size(), EPIDMC_E_RANGE, "layer material");
        REQUIRE(std::isfinite(layers[l].thickness) && layers[l].thickness > 0, EPIDMC_E_ARG, "layer thickness > 0");
        REQUIRE(std::isfinite(layers[l].density) && layers[l].density >= 0, EPIDMC_E_ARG, "layer density >= 0");
    }
    c->layers.assign(layers, layers + nl);
    c->scoring = scoring;
    c->front_z = front_z;
    c->npx_u = npx_u; c->npx_v = npx_v;
    c->pitch_u = pitch_u; c->pitch_v = pitch_v;
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_source_spectrum(epidmc_ctx *c, const float *edges, const float *w, int nbins, const epidmc_beam *beam)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(edges && w && beam && nbins >= 1 && nbins <= 65536, EPIDMC_E_ARG, "spectrum arrays");
    REQUIRE(beam->kind == 0 || beam->kind == 1, EPIDMC_E_ARG, "beam kind 0 (parallel) or 1 (point)");
    REQUIRE(finite3(beam->src) && std::isfinite(beam->iso_z), EPIDMC_E_ARG, "beam geometry must be finite");
    REQUIRE(beam->kind == 0 || beam->iso_z != beam->src[2], EPIDMC_E_ARG, "point source on its aperture plane");
    double tot = 0;
    for (int i = 0; i < nbins; ++i) {
        REQUIRE(std::isfinite(w[i]) && w[i] >= 0, EPIDMC_E_ARG, "spectrum weights must be >= 0");
        tot += w[i];
    }
    REQUIRE(tot > 0, EPIDMC_E_ARG, "spectrum weights sum to zero");
    for (int i = 0; i <= nbins; ++i) {
        REQUIRE(std::isfinite(edges[i]), EPIDMC_E_ARG, "bin edges must be finite");
        if (i) REQUIRE(edges[i] >= edges[i - 1], EPIDMC_E_ARG, "bin edges must not decrease");
    }
    REQUIRE(edges[nbins] <= 50.0f, EPIDMC_E_RANGE, "energies above 50 MeV are not supported");
    c->edges.assign(edges, edges + nbins + 1);
    c->weights.assign(w, w + nbins);
    c->beam = *beam;
    c->have_spectrum = true;
    c->phsp.clear();
    c->n_phsp = 0;
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_source_phsp(epidmc_ctx *c, const epidmc_particle *p, uint64_t n)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(p && n >= 1 && n <= (1ull << 28), EPIDMC_E_ARG, "phase-space list");
    std::vector<float> v(8 * n);
    for (uint64_t i = 0; i < n; ++i) {
        const epidmc_particle &q = p[i];
        REQUIRE(q.type == 0 || q.type == 1, EPIDMC_E_ARG, "phase-space particles are photons (0) or electrons (1)");
        REQUIRE(std::isfinite(q.x) && std::isfinite(q.y) && std::isfinite(q.z) && std::isfinite(q.E), EPIDMC_E_ARG,
                "phase-space values must be finite");
        REQUIRE(q.E > 0 && q.E <= 50.0f, EPIDMC_E_RANGE, "phase-space energy in (0, 50] MeV");
        const double nn = std::sqrt((double)q.u * q.u + (double)q.v * q.v + (double)q.w * q.w);
        REQUIRE(std::fabs(nn - 1.0) < 1e-3, EPIDMC_E_ARG, "phase-space directions must be unit vectors");
        const float f[8] = {q.x, q.y, q.z, (float)(q.u / nn), (float)(q.v / nn), (float)(q.w / nn), q.E, (float)q.type};
        std::memcpy(&v[8 * i], f, sizeof f);
    }
    c->phsp.swap(v);
    c->n_phsp = n;
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_segments(epidmc_ctx *c, int n_seg, int n_pairs, float leaf_w, float y0, const float *a,
                                  const float *b, const uint64_t *n_hist)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(n_seg >= 1 && n_seg <= EPIDMC_MAX_SEGMENTS && n_pairs >= 1 && n_pairs <= 1024 && a && b, EPIDMC_E_ARG,
            "segments: 1..256 segments, 1..1024 leaf pairs");
    REQUIRE(std::isfinite(leaf_w) && leaf_w > 0 && std::isfinite(y0), EPIDMC_E_ARG, "leaf width > 0");
    REQUIRE(n_seg == 1 || n_hist, EPIDMC_E_ARG, "several segments need history counts");
    for (int s = 0; s < n_seg; ++s) {
        double open = 0;
        for (int k = 0; k < n_pairs; ++k) {
            const float lo = a[s * n_pairs + k], hi = b[s * n_pairs + k];
            REQUIRE(std::isfinite(lo) && std::isfinite(hi) && lo <= hi, EPIDMC_E_ARG, "leaf positions need a <= b");
            open += hi - lo;
        }
        REQUIRE(open > 0 || (n_seg > 1 && n_hist[s] == 0), EPIDMC_E_ARG, "a segment with histories has no open area");
    }
    uint64_t tot = 0;
    if (n_seg > 1)
        for (int s = 0; s < n_seg; ++s) {
            REQUIRE(tot + n_hist[s] >= tot, EPIDMC_E_RANGE, "segment history counts overflow 64 bits");
            tot += n_hist[s];
        }
    c->n_seg = n_seg;
    c->n_pairs = n_pairs;
    c->leaf_w = leaf_w;
    c->y0 = y0;
    c->ap_a.assign(a, a + (size_t)n_seg * n_pairs);
    c->ap_b.assign(b, b + (size_t)n_seg * n_pairs);
    c->seg_hist.assign(n_seg, 0);
    if (n_seg > 1) std::copy(n_hist, n_hist + n_seg, c->seg_hist.begin());
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_tally(epidmc_ctx *c, epidmc_tally_mode mode, int batches, uint64_t max_chunk)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(mode >= EPIDMC_TALLY_FP64 && mode <= EPIDMC_TALLY_KAHAN32, EPIDMC_E_ARG, "unknown tally mode");
    REQUIRE(batches >= 2 && batches <= 1 << 20, EPIDMC_E_ARG, "batches per run in [2, 2^20]");
    REQUIRE(max_chunk >= 1024 && max_chunk <= (1ull << 27), EPIDMC_E_RANGE, "chunk in [1024, 2^27] histories");
    c->tally_mode = (int)mode;
    c->batches = batches;
    c->max_chunk = max_chunk;
    unbind(c);
    return EPIDMC_OK;
}

epidmc_status epidmc_set_profiling(epidmc_ctx *c, int enable)
{
    if (!c) return EPIDMC_E_ARG;
    if (enable && !c->ev[0][0]) {
        HIPCHK(hipSetDevice(c->device));
        for (int b = 0; b < 2; ++b)
            for (int k = 0; k < NQ; ++k) HIPCHK(hipEventCreate(&c->ev[b][k]));
        for (int p = 0; p < MAX_DEV_PASSES; ++p)
            for (int b = 0; b < 2; ++b)
                for (int k = 0; k < NQ; ++k) HIPCHK(hipEventCreate(&c->dev_ev[p][b][k]));
    }
    c->prof = enable ? 1 : 0;
    return EPIDMC_OK;
}

epidmc_status epidmc_set_passes(epidmc_ctx *c, int device_passes, int items_per_lane)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(device_passes >= -1 && device_passes <= MAX_DEV_PASSES, EPIDMC_E_ARG, "device passes in [-1, 24]");
    REQUIRE(items_per_lane >= 1 && items_per_lane <= 64, EPIDMC_E_ARG, "items per lane in [1, 64]");
    c->dev_passes = device_passes;
    c->ipl = items_per_lane;
    return EPIDMC_OK;
}

epidmc_status epidmc_set_graph(epidmc_ctx *c, int enable, int passes)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(passes >= 0 && passes <= MAX_DEV_PASSES, EPIDMC_E_ARG, "graph passes in [0, 24]");
    REQUIRE(!enable || (c->tally_mode != 2 && !c->diag), EPIDMC_E_ARG,
            "graph runs need the FP64 or fixed-point tally and diagnostics off");
    drop_graph(c);
    c->graph = enable ? 1 : 0;
    c->graph_passes = passes;
    return EPIDMC_OK;
}

epidmc_status epidmc_set_diagnostics(epidmc_ctx *c, int enable)
{
    if (!c) return EPIDMC_E_ARG;
    c->diag = enable ? 1 : 0;
    unbind(c);
    return EPIDMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------------
static epidmc_status model_ready(epidmc_ctx *c)
{
    REQUIRE(!c->mats.empty(), EPIDMC_E_NOT_READY, "materials not set");
    REQUIRE(c->nx > 0, EPIDMC_E_NOT_READY, "phantom not set");
    REQUIRE(!c->layers.empty(), EPIDMC_E_NOT_READY, "EPID not set");
    REQUIRE(c->have_spectrum || c->n_phsp > 0, EPIDMC_E_NOT_READY, "source not set");
    REQUIRE(c->n_phsp > 0 || c->n_seg > 0, EPIDMC_E_NOT_READY, "aperture segments not set");
    for (size_t i = 0; i < c->vmat.size(); ++i)
        REQUIRE(c->vmat[i] < c->mats.size(), EPIDMC_E_RANGE, "voxel material not in the material table");
    for (auto &l : c->layers) REQUIRE(l.material < (int)c->mats.size(), EPIDMC_E_RANGE, "layer material not in the table");
    // distinct phantom materials
    bool seen[EPIDMC_MAX_MATERIALS] = {false};
    for (uint8_t m : c->vmat) seen[m] = true;
    int k = 0;
    for (int m = 0; m < EPIDMC_MAX_MATERIALS; ++m) {
        c->slot_of_mat[m] = -1;
        if (seen[m]) c->slot_of_mat[m] = k++;
    }
    REQUIRE(k <= MAX_PMAT, EPIDMC_E_RANGE, "at most 4 distinct materials in one phantom");
    return EPIDMC_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout make_layout(const epidmc_ctx *c)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](Region &r, size_t bytes) { r.off = off; r.bytes = bytes; off = align256(off + bytes); };
    const size_t nvox = (size_t)c->nx * c->ny * c->nz;
    const size_t npix = (size_t)c->npx_u * c->npx_v;
    const uint64_t H = c->max_chunk;
    L.chunk = H;
    L.cap[QGP] = (uint32_t)(H + 4096);
    L.cap[QEP] = (uint32_t)(4 * H + 4096);
    L.cap[QGE] = (uint32_t)(2 * H + 4096);
    L.cap[QEE] = (uint32_t)(2 * H + 4096);
    // A pass of n items runs on about n / (WG * ITEMS_PER_LANE) workgroups, i.e. n / 128
    // waves, so its waves use min(n / 128, NSEG) home segments.  Every segment therefore holds
    // at least MIN_SEGCAP particles: with fewer than NSEG segments in use, a segment takes the
    // appends of about 128 items (at most a few thousand particles); with all in use, 1/NSEG of
    // the queue's capacity.
    constexpr uint32_t MIN_SEGCAP = 16384;
    for (int k = 0; k < NQ; ++k) {
        L.segcap[k] = std::max<uint32_t>((L.cap[k] + NSEG - 1) / NSEG, MIN_SEGCAP);
        if (c->q_override[k]) L.segcap[k] = c->q_override[k];
        L.cap[k] = L.segcap[k] * NSEG;
    }
    L.rec_cap = c->tally_mode == 2 ? (uint32_t)(8 * H + 4096) : 0;
    L.ring = std::min(c->batches, MAX_SLOTS);
    const int nbins = std::max<int>(1, (int)c->weights.size());
    const size_t nap = (size_t)std::max(1, c->n_seg) * std::max(1, c->n_pairs);
    take(L.vox, nvox * 4);
    take(L.ph_tab, (size_t)(MAX_PMAT + MAX_LAYERS) * 3 * NB_PH * 4);
    take(L.ph_maj, NB_PH * 4);
    take(L.ph_mu4, NB_PH * 16);
    take(L.ph_fr, (size_t)MAX_PMAT * NB_PH * 8);
    take(L.el_tab, (size_t)(MAX_PMAT + MAX_LAYERS) * 3 * NB_EL * 4);
    take(L.sp_lo, nbins * 4);
    take(L.sp_hi, nbins * 4);
    take(L.sp_prob, nbins * 4);
    take(L.sp_alias, nbins * 4);
    take(L.ap_a, nap * 4);
    take(L.ap_b, nap * 4);
    take(L.ap_prob, nap * 4);
    take(L.ap_alias, nap * 4);
    take(L.seg_end, (size_t)std::max(1, c->n_seg) * 8);
    take(L.phsp, std::max<size_t>(1, c->n_phsp) * 32);
    take(L.ctl, CTL_BYTES);
    take(L.segc, 3 * SEG_SET * 4);   // segment fill counters of the two buffer sets, consume heads
    size_t qb = 0;
    for (int k = 0; k < NQ; ++k) qb += (size_t)L.cap[k] * 48;
    take(L.queues, 2 * qb);
    take(L.img, (size_t)L.ring * npix * 8);
    take(L.sum, npix * 8);
    take(L.sum2, npix * 8);
    take(L.led, c->diag ? H * 8 : 8);
    take(L.ein, c->diag ? H * 8 : 8);
    const size_t nimg = (size_t)L.ring * npix;
    take(L.rec_pix, (size_t)L.rec_cap * 4 + 4);
    take(L.rec_e, (size_t)L.rec_cap * 4 + 4);
    take(L.k_count, c->tally_mode == 2 ? nimg * 4 : 4);
    take(L.k_cursor, c->tally_mode == 2 ? nimg * 4 : 4);
    take(L.k_bsum, c->tally_mode == 2 ? (nimg / 1024 + 2) * 4 : 4);
    take(L.k_sorted, (size_t)L.rec_cap * 4 + 4);
    L.total = off;
    return L;
}

extern "C" epidmc_status epidmc_workspace_size(epidmc_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return EPIDMC_E_ARG;
    epidmc_status s = model_ready(c);
    if (s != EPIDMC_OK) return s;
    *bytes = make_layout(c).total;
    return EPIDMC_OK;
}

// ---------------------------------------------------------------------------------
// binding: build tables and upload
// ---------------------------------------------------------------------------------
extern "C" epidmc_status epidmc_bind_workspace(epidmc_ctx *c, void *dev, size_t bytes, void *stream)
{
    if (!c) return EPIDMC_E_ARG;
    epidmc_status st = model_ready(c);
    if (st != EPIDMC_OK) return st;
    REQUIRE(dev && ((uintptr_t)dev % 256) == 0, EPIDMC_E_WORKSPACE, "workspace must be 256-byte aligned");
    const Layout L = make_layout(c);
    REQUIRE(bytes >= L.total, EPIDMC_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total) + " bytes");
    HIPCHK(hipSetDevice(c->device));
    drop_graph(c);   // a captured run holds the previous workspace's addresses
    c->have_rows = false;   // pass statistics of another model
    c->last_passes = 0;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)dev;

    // energy grids
    float emax = 0.52f;
    for (float e : c->edges) emax = std::max(emax, e);
    for (uint64_t i = 0; i < c->n_phsp; ++i) emax = std::max(emax, c->phsp[8 * i + 6]);
    const double ehi = 1.02 * emax;
    const double ph0 = std::log((double)c->pcut), phd = (std::log(ehi) - ph0) / (NB_PH - 1);
    const double el0 = std::log(0.5 * (double)c->ecut), eld = (std::log(ehi) - el0) / (NB_EL - 1);

    // phantom packing: density bits with the two low bits replaced by the material slot
    const size_t nvox = c->vmat.size();
    std::vector<uint32_t> vox(nvox);
    float rho_max[MAX_PMAT] = {0, 0, 0, 0};
    int mat_of_slot[MAX_PMAT] = {0, 0, 0, 0};
    int nslot = 0;
    for (int m = 0; m < EPIDMC_MAX_MATERIALS; ++m)
        if (c->slot_of_mat[m] >= 0) { mat_of_slot[c->slot_of_mat[m]] = m; nslot = std::max(nslot, c->slot_of_mat[m] + 1); }
    for (size_t i = 0; i < nvox; ++i) {
        uint32_t bits;
        std::memcpy(&bits, &c->vrho[i], 4);
        const uint32_t slot = (uint32_t)c->slot_of_mat[c->vmat[i]];
        vox[i] = (bits & ~3u) | slot;
        float r;
        const uint32_t rb = bits & ~3u;
        std::memcpy(&r, &rb, 4);
        rho_max[slot] = std::max(rho_max[slot], r);
    }

    // tables
    std::vector<float> ph_tab((size_t)(MAX_PMAT + MAX_LAYERS) * 3 * NB_PH, 0.0f);
    std::vector<float> el_tab((size_t)(MAX_PMAT + MAX_LAYERS) * 3 * NB_EL, 0.0f);
    std::vector<float> maj(NB_PH, 0.0f);
    float x0[MAX_PMAT + MAX_LAYERS] = {0};
    auto build_slot = [&](int slot, int mat) {
        const MatDerived d = derive(c->mats[mat]);
        build_photon_table(d, c->mask, ph0, phd, &ph_tab[(size_t)slot * 3 * NB_PH]);
        build_electron_table(d, c->mask, el0, eld, &el_tab[(size_t)slot * 3 * NB_EL]);
        x0[slot] = (float)d.x0;
    };
    for (int s2 = 0; s2 < nslot; ++s2) build_slot(s2, mat_of_slot[s2]);
    for (size_t l = 0; l < c->layers.size(); ++l) build_slot(MAX_PMAT + (int)l, c->layers[l].material);
    for (int i = 0; i < NB_PH; ++i) {
        double m = 0;
        for (int s2 = 0; s2 < nslot; ++s2) m = std::max(m, (double)rho_max[s2] * ph_tab[(size_t)s2 * 3 * NB_PH + i]);
        maj[i] = (float)(m * (1.0 + 1e-5));   // margin over the FP32 rounding of rho * mu
    }
    // the Woodcock kernel's packed copies: per node the four slots' mu/rho in one 16-byte word,
    // per slot and node the two cumulative process fractions in one 8-byte word
    std::vector<float> mu4((size_t)NB_PH * 4, 0.0f), fr((size_t)MAX_PMAT * NB_PH * 2, 0.0f);
    for (int s2 = 0; s2 < nslot; ++s2)
        for (int i = 0; i < NB_PH; ++i) {
            const float *t = &ph_tab[(size_t)s2 * 3 * NB_PH];
            mu4[(size_t)i * 4 + s2] = t[i];
            fr[((size_t)s2 * NB_PH + i) * 2] = t[NB_PH + i];
            fr[((size_t)s2 * NB_PH + i) * 2 + 1] = t[2 * NB_PH + i];
        }

    // source
    const int nbins = std::max<int>(1, (int)c->weights.size());
    std::vector<float> sp_lo(nbins, 0), sp_hi(nbins, 0), sp_prob(nbins, 1), ap_prob, ap_a, ap_b;
    std::vector<int> sp_alias(nbins, 0), ap_alias;
    if (!c->weights.empty()) {
        std::vector<double> w(c->weights.begin(), c->weights.end());
        build_alias(w, sp_prob, sp_alias);
        for (int i = 0; i < nbins; ++i) { sp_lo[i] = c->edges[i]; sp_hi[i] = c->edges[i + 1]; }
    }
    const int nseg = std::max(1, c->n_seg), npair = std::max(1, c->n_pairs);
    ap_a.assign((size_t)nseg * npair, 0.0f);
    ap_b.assign((size_t)nseg * npair, 0.0f);
    ap_prob.assign((size_t)nseg * npair, 1.0f);
    ap_alias.assign((size_t)nseg * npair, 0);
    std::vector<unsigned long long> seg_end(nseg, ~0ull);
    if (c->n_seg > 0) {
        ap_a = c->ap_a;
        ap_b = c->ap_b;
        unsigned long long cum = 0;
        for (int s2 = 0; s2 < c->n_seg; ++s2) {
            std::vector<double> wv(c->n_pairs);
            for (int k = 0; k < c->n_pairs; ++k) wv[k] = (double)c->ap_b[s2 * c->n_pairs + k] - c->ap_a[s2 * c->n_pairs + k];
            std::vector<float> pr;
            std::vector<int> al;
            build_alias(wv, pr, al);
            std::copy(pr.begin(), pr.end(), ap_prob.begin() + (size_t)s2 * c->n_pairs);
            std::copy(al.begin(), al.end(), ap_alias.begin() + (size_t)s2 * c->n_pairs);
            cum += c->seg_hist[s2];
            seg_end[s2] = c->n_seg > 1 ? cum : ~0ull;
        }
    }

    // uploads
    auto up = [&](const Region &r, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(w + r.off, src, n, hipMemcpyHostToDevice, s);
    };
    HIPCHK(up(L.vox, vox.data(), nvox * 4));
    HIPCHK(up(L.ph_tab, ph_tab.data(), ph_tab.size() * 4));
    HIPCHK(up(L.ph_maj, maj.data(), maj.size() * 4));
    HIPCHK(up(L.ph_mu4, mu4.data(), mu4.size() * 4));
    HIPCHK(up(L.ph_fr, fr.data(), fr.size() * 4));
    HIPCHK(up(L.el_tab, el_tab.data(), el_tab.size() * 4));
    HIPCHK(up(L.sp_lo, sp_lo.data(), nbins * 4));
    HIPCHK(up(L.sp_hi, sp_hi.data(), nbins * 4));
    HIPCHK(up(L.sp_prob, sp_prob.data(), nbins * 4));
    HIPCHK(up(L.sp_alias, sp_alias.data(), nbins * 4));
    HIPCHK(up(L.ap_a, ap_a.data(), ap_a.size() * 4));
    HIPCHK(up(L.ap_b, ap_b.data(), ap_b.size() * 4));
    HIPCHK(up(L.ap_prob, ap_prob.data(), ap_prob.size() * 4));
    HIPCHK(up(L.ap_alias, ap_alias.data(), ap_alias.size() * 4));
    HIPCHK(up(L.seg_end, seg_end.data(), seg_end.size() * 8));
    if (c->n_phsp) HIPCHK(up(L.phsp, c->phsp.data(), c->phsp.size() * 4));
    HIPCHK(launch_zero(w + L.ctl.off, L.ctl.bytes, s));
    HIPCHK(launch_zero(w + L.img.off, L.img.bytes, s));
    HIPCHK(launch_zero(w + L.sum.off, L.sum.bytes, s));
    HIPCHK(launch_zero(w + L.sum2.off, L.sum2.bytes, s));
    HIPCHK(launch_zero(w + L.led.off, L.led.bytes, s));
    HIPCHK(hipStreamSynchronize(s));   // host vectors go out of scope

    // parameters
    Params &P = c->P;
    P = Params{};
    char *q = w + L.queues.off;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < NQ; ++k) {
            Queue &Q = c->qs[b][k];
            const size_t n = L.cap[k];
            uint4 **fp[3] = {&Q.a, &Q.b, &Q.c};
            for (int f = 0; f < 3; ++f) { *fp[f] = (uint4 *)q; q += n * 16; }
        }
    for (int k = 0; k < NQ; ++k) P.segcap[k] = L.segcap[k];
    char *ctl = w + L.ctl.off;
    P.cnt = (uint32_t *)(ctl + CTL_CNT);
    P.heads = nullptr;   // set per pass by run_chunk (segment counters)
    P.err = (uint32_t *)(ctl + CTL_ERR);
    P.stats = (unsigned long long *)(ctl + CTL_STATS);
    P.nx = c->nx; P.ny = c->ny; P.nz = c->nz;
    P.dx = c->spacing[0]; P.dy = c->spacing[1]; P.dz = c->spacing[2];
    P.idx = 1.0f / P.dx; P.idy = 1.0f / P.dy; P.idz = 1.0f / P.dz;
    P.Lx = (float)((double)c->nx * c->spacing[0]);
    P.Ly = (float)((double)c->ny * c->spacing[1]);
    P.Lz = (float)((double)c->nz * c->spacing[2]);
    P.ox = c->origin[0]; P.oy = c->origin[1]; P.oz = c->origin[2];
    P.chord = P.Lx + P.Ly + P.Lz + 1.0f;
    P.ddx = c->spacing[0]; P.ddy = c->spacing[1]; P.ddz = c->spacing[2];
    P.iddx = 1.0 / P.ddx; P.iddy = 1.0 / P.ddy; P.iddz = 1.0 / P.ddz;
    P.vox = (const uint32_t *)(w + L.vox.off);
    P.nl = (int)c->layers.size();
    P.scoring = c->scoring;
    double z = 0;
    P.zl[0] = 0.0f;
    for (int l = 0; l < P.nl; ++l) {
        z += c->layers[l].thickness;
        P.zl[l + 1] = (float)z;
        P.lrho[l] = c->layers[l].density;
    }
    for (int l = P.nl + 1; l <= MAX_LAYERS; ++l) P.zl[l] = (float)z;
    P.zback = (float)z;
    P.front_z = c->front_z;
    P.hx = (float)(0.5 * c->npx_u * (double)c->pitch_u);
    P.hy = (float)(0.5 * c->npx_v * (double)c->pitch_v);
    P.npx_u = c->npx_u; P.npx_v = c->npx_v;
    P.pitch_u = c->pitch_u; P.pitch_v = c->pitch_v;
    P.ipu = 1.0f / c->pitch_u; P.ipv = 1.0f / c->pitch_v;
    P.s_pix = 0.5f * std::min(c->pitch_u, c->pitch_v);
    P.ph_to_epid_z = (float)((double)c->front_z - (double)c->origin[2]);
    P.ph_tab = (const float *)(w + L.ph_tab.off);
    P.ph_maj = (const float *)(w + L.ph_maj.off);
    P.ph_mu4 = (const float4 *)(w + L.ph_mu4.off);
    P.ph_fr = (const float2 *)(w + L.ph_fr.off);
    for (int s2 = 0; s2 < MAX_PMAT; ++s2) P.rmaj[s2] = (float)((double)rho_max[s2] * (1.0 + 1e-5));
    P.el_tab = (const float *)(w + L.el_tab.off);
    P.ph_lnE0 = (float)ph0; P.ph_idl = (float)(1.0 / phd);
    P.el_lnT0 = (float)el0; P.el_idl = (float)(1.0 / eld);
    for (int i = 0; i < MAX_PMAT + MAX_LAYERS; ++i) P.el_x0[i] = x0[i];
    P.nmat_ph = nslot;
    P.coupled = c->coupled;
    P.mask = c->mask;
    P.pcut = c->pcut;
    P.ecut = c->ecut;
    P.beam_kind = c->beam.kind;
    for (int a = 0; a < 3; ++a) P.src[a] = c->beam.src[a];
    P.iso_z = c->beam.iso_z;
    P.nbins = nbins;
    P.sp_lo = (const float *)(w + L.sp_lo.off);
    P.sp_hi = (const float *)(w + L.sp_hi.off);
    P.sp_prob = (const float *)(w + L.sp_prob.off);
    P.sp_alias = (const int *)(w + L.sp_alias.off);
    P.n_seg = nseg;
    P.n_pairs = npair;
    P.leaf_w = c->leaf_w;
    P.y0 = c->y0;
    P.ap_a = (const float *)(w + L.ap_a.off);
    P.ap_b = (const float *)(w + L.ap_b.off);
    P.ap_prob = (const float *)(w + L.ap_prob.off);
    P.ap_alias = (const int *)(w + L.ap_alias.off);
    P.seg_end = (const unsigned long long *)(w + L.seg_end.off);
    P.phsp = c->n_phsp ? (const float *)(w + L.phsp.off) : nullptr;
    P.n_phsp = c->n_phsp;
    P.tally_mode = c->tally_mode;
    P.npix = (uint32_t)((size_t)c->npx_u * c->npx_v);
    P.img = w + L.img.off;
    P.rec_pix = (uint32_t *)(w + L.rec_pix.off);
    P.rec_e = (float *)(w + L.rec_e.off);
    P.rec_cap = L.rec_cap;
    P.sum = (double *)(w + L.sum.off);
    P.sum2 = (double *)(w + L.sum2.off);
    P.diag = c->diag;
    P.led = (double *)(w + L.led.off);
    P.ein = (double *)(w + L.ein.off);
    P.key0 = (uint32_t)c->seed;
    P.key1 = (uint32_t)(c->seed >> 32);
    P.run_batches = 1;
    P.run_n = 1;

    // workgroups per CU each transport kernel can keep resident
    for (int k = 0; k < NQ; ++k) {
        const size_t lds = lds_bytes(k, P);
        c->occ[k] = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / std::max<size_t>(lds, 1)));
    }
    c->ws = w;
    c->ws_bytes = bytes;
    c->lay = L;
    c->bound = true;
    c->n_total = 0;
    c->b_total = 0;
    c->launches = 0;
    c->queue_peak = 0;
    return EPIDMC_OK;
}

// ---------------------------------------------------------------------------------
// run
// ---------------------------------------------------------------------------------
static epidmc_status check_error_word(epidmc_ctx *c, uint32_t e)
{
    if (e & ERR_NAN) return fail(c, EPIDMC_E_NAN, "non-finite particle energy on the device");
    if (e & ERR_QUEUE) return fail(c, EPIDMC_E_OVERFLOW, "particle queue overflow: lower max_chunk_histories");
    if (e & ERR_STEPS) return fail(c, EPIDMC_E_OVERFLOW, "electron step limit exceeded");
    if (e & ERR_FIXED) return fail(c, EPIDMC_E_OVERFLOW, "fixed-point tally overflow");
    if (e & ERR_SAMPLE) return fail(c, EPIDMC_E_OVERFLOW, "Klein-Nishina sample not accepted within the draw limit");
    return EPIDMC_OK;
}

// histories of variance batch b of a run [first, first+n) split into B batches: batch of h
// is (h - first) * B / n, so batch b starts at first + ceil(b n / B)
static uint64_t batch_start(uint64_t first, uint64_t n, int B, uint64_t b)
{
    return first + (b * n + (uint64_t)B - 1) / (uint64_t)B;
}

static epidmc_status kind_streams(epidmc_ctx *c)
{
    if (c->go) return EPIDMC_OK;
    for (int k = 0; k < NQ - 1; ++k) {
        HIPCHK(hipStreamCreateWithFlags(&c->ks[k], hipStreamNonBlocking));   // default priority
        HIPCHK(hipEventCreateWithFlags(&c->done[k], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&c->go, hipEventDisableTiming));
    return EPIDMC_OK;
}

// Launch one pass's kernels: each kind on its own stream (the last on the run stream), all
// starting together once the pass-start kernel has run, the run stream waiting for the others
// afterwards.  `blocks[k] == 0` skips a kind; `ev` (or null) brackets each launch for profiling.
static epidmc_status launch_pass(epidmc_ctx *c, const Params &P, const unsigned *blocks, hipEvent_t (*ev)[NQ],
                                 hipStream_t s)
{
    HIPCHK(hipEventRecord(c->go, s));
    for (int k = 0; k < NQ; ++k) {
        if (!blocks[k]) continue;
        const bool own = k < NQ - 1;
        hipStream_t ks = own ? c->ks[k] : s;
        if (own) HIPCHK(hipStreamWaitEvent(ks, c->go, 0));
        if (ev) HIPCHK(hipEventRecord(ev[0][k], ks));
        HIPCHK(launch_transport(k, P, blocks[k], ks));
        if (ev) HIPCHK(hipEventRecord(ev[1][k], ks));
        if (own) HIPCHK(hipEventRecord(c->done[k], ks));
    }
    for (int k = 0; k < NQ - 1; ++k)
        if (blocks[k]) HIPCHK(hipStreamWaitEvent(s, c->done[k], 0));
    return EPIDMC_OK;
}

// One chunk of histories [h0, h1): the source, then queue passes until every queue is empty.
// The first K passes are device-driven: every kind is launched at its resident grid size and
// its blocks beyond the queue's need leave at once (gated_off), so no pass waits for the host;
// the pass-start kernel keeps each pass's totals, which the host reads once afterwards.  The
// passes after that are host-driven (one readback each, grids sized from the totals).  In a
// graph capture (`capture`) the chunk runs exactly K device-driven passes and a last
// pass-start kernel that flags any queue still holding particles.
static epidmc_status run_chunk(epidmc_ctx *c, uint64_t h0, uint64_t h1, hipStream_t s, bool capture = false,
                               int chunk = 0)
{
    {
        const epidmc_status st = kind_streams(c);
        if (st != EPIDMC_OK) return st;
    }
    Params P = c->P;
    P.h0 = h0;
    P.h1 = h1;
    P.ipl = c->ipl;
    P.gated = 0;
    // history ids of 2^32 and above: the counter's history word holds the low 32 bits and
    // the high word selects the key (odd multipliers keep distinct high words distinct);
    // a chunk never spans a 2^32 boundary, so one key serves the whole chunk
    const uint32_t hi = (uint32_t)(h0 >> 32);
    P.key0 ^= hi * 0x9E3779B9u;
    P.key1 ^= hi * 0x85EBCA6Bu;
    uint32_t *cnt = P.cnt;
    uint32_t *seg = (uint32_t *)(c->ws + c->lay.segc.off);   // [set A, set B, heads][NQ][NSEG] x CSTRIDE
    uint32_t *hist = (uint32_t *)(c->ws + c->lay.ctl.off + CTL_PASSHIST);
    HIPCHK(launch_zero(cnt, 64, s));
    HIPCHK(launch_zero(seg, 3 * SEG_SET * 4, s));
    // the source appends into buffer set 0
    auto use = [&](int cur) {
        for (int k = 0; k < NQ; ++k) { P.in[k] = c->qs[cur][k]; P.out[k] = c->qs[1 - cur][k]; }
        P.cnt_in = seg + cur * SEG_SET;
        P.cnt_out = seg + (1 - cur) * SEG_SET;
        P.heads = seg + 2 * SEG_SET;
    };
    use(1);
    HIPCHK(launch_source(P, s));
    ++c->launches;
    int cur = 0;
    const int K = std::min(capture ? c->graph_passes : (c->dev_passes < 0 ? c->last_passes : c->dev_passes),
                           MAX_DEV_PASSES);
    const bool prof = c->prof && !capture;
    int pass = 0;
    // device-driven passes: pass-start (totals kept per pass), then every kind, gated on the device
    for (; pass < K; ++pass) {
        HIPCHK(launch_pass_start(P, seg + cur * SEG_SET, cnt, seg + (1 - cur) * SEG_SET, seg + 2 * SEG_SET, SEG_SET, s,
                                 hist + pass * (NQ + 1)));
        use(cur);
        P.gated = 1;
        // grids sized from the previous chunk's totals of the same pass, with headroom (a queue
        // that holds more than its grid was sized for is still drained, by fewer waves); a kind
        // that was empty gets one workgroup, which leaves at once when its queue is empty again
        unsigned blocks[NQ];
        for (int k = 0; k < NQ; ++k) {
            const uint64_t full = (uint64_t)c->n_cu * c->occ[k], per = (uint64_t)WG * c->ipl;
            const uint64_t want = c->have_rows ? (c->prev_rows[pass][k] + c->prev_rows[pass][k] / 4 + per - 1) / per : full;
            blocks[k] = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, full));
        }
        const epidmc_status st = launch_pass(c, P, blocks, prof ? c->dev_ev[pass] : nullptr, s);
        if (st != EPIDMC_OK) return st;
        P.gated = 0;
        cur = 1 - cur;
    }
    if (capture) {
        // what the queues still hold after the last captured pass, kept per chunk: the host
        // checks after the replay that every queue was empty
        HIPCHK(launch_pass_start(P, seg + cur * SEG_SET, cnt, seg + (1 - cur) * SEG_SET, seg + 2 * SEG_SET, SEG_SET, s,
                                 (uint32_t *)(c->ws + c->lay.ctl.off + CTL_LEFT) + chunk * (NQ + 1)));
        return EPIDMC_OK;
    }
    bool timed[NQ] = {false, false, false, false};
    int nonempty = -1;   // the first pass that found every queue empty
    uint32_t rows[MAX_DEV_PASSES][NQ] = {};
    for (; pass < 100000; ++pass) {
        // the input set's totals and the error word in one readback; the kernel also clears
        // the other set's fill counters and the consume heads for this pass (the previous
        // pass, which used them, has ended: the run stream waited for it)
        HIPCHK(launch_pass_start(P, seg + cur * SEG_SET, cnt, seg + (1 - cur) * SEG_SET, seg + 2 * SEG_SET, SEG_SET, s,
                                 nullptr));
        HIPCHK(hipMemcpyAsync(c->host, cnt, (NQ + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        if (pass == K && K > 0)
            HIPCHK(hipMemcpyAsync(c->host + 16, hist, (size_t)K * (NQ + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (pass == K && K > 0) {
            // what the device-driven passes held, and their profiled kernels
            for (int p = 0; p < K; ++p) {
                const uint32_t *row = c->host + 16 + p * (NQ + 1);
                bool any = false;
                for (int k = 0; k < NQ; ++k) {
                    rows[p][k] = row[k];
                    if (!row[k]) continue;
                    any = true;
                    ++c->launches;
                    c->queue_peak = std::max<uint64_t>(c->queue_peak, row[k]);
                    if (prof) {
                        float ms = 0.0f;
                        HIPCHK(hipEventElapsedTime(&ms, c->dev_ev[p][0][k], c->dev_ev[p][1][k]));
                        c->kernel_ms[k] += ms;
                        ++c->kernel_launches[k];
                    }
                }
                if (!any && nonempty < 0) nonempty = p;
            }
        }
        for (int k = 0; k < NQ; ++k)
            if (timed[k]) {
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, c->ev[0][k], c->ev[1][k]));
                c->kernel_ms[k] += ms;
                ++c->kernel_launches[k];
                timed[k] = false;
            }
        uint32_t n[NQ];
        std::memcpy(n, c->host, sizeof n);
        if (pass < MAX_DEV_PASSES) std::memcpy(rows[pass], n, sizeof n);
        if (c->host[NQ] & (ERR_QUEUE | ERR_NAN | ERR_STEPS | ERR_SAMPLE)) return check_error_word(c, c->host[NQ]);
        bool any = false;
        for (int k = 0; k < NQ; ++k) {
            any |= n[k] > 0;
            c->queue_peak = std::max<uint64_t>(c->queue_peak, n[k]);
        }
        if (!any) {
            if (nonempty < 0) nonempty = pass;
            break;
        }
        use(cur);
        unsigned blocks[NQ];
        for (int k = 0; k < NQ; ++k) {
            const uint64_t per_block = (uint64_t)WG * c->ipl;
            const uint64_t want = (n[k] + per_block - 1) / per_block;
            blocks[k] = n[k] ? (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)c->n_cu * c->occ[k])) : 0u;
            if (blocks[k]) {
                ++c->launches;
                timed[k] = prof;
            }
        }
        const epidmc_status st = launch_pass(c, P, blocks, prof ? c->ev : nullptr, s);
        if (st != EPIDMC_OK) return st;
        cur = 1 - cur;
    }
    c->last_passes = nonempty;
    std::memcpy(c->prev_rows, rows, sizeof rows);
    c->have_rows = true;
    if (c->tally_mode == 2) {
        HIPCHK(hipMemcpyAsync(c->host, cnt + 3 * NQ, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const uint32_t nrec = std::min(c->host[0], c->lay.rec_cap);
        c->last_nrec = nrec;
        const uint32_t nimg = (uint32_t)((size_t)c->lay.ring * P.npix);
        HIPCHK(launch_kahan_reduce(P, nrec, nimg, (uint32_t *)(c->ws + c->lay.k_count.off),
                                   (uint32_t *)(c->ws + c->lay.k_cursor.off), (uint32_t *)(c->ws + c->lay.k_bsum.off),
                                   (float *)(c->ws + c->lay.k_sorted.off), s));
        HIPCHK(launch_zero(cnt + 3 * NQ, 4, s));
    }
    if (c->diag) {
        HIPCHK(launch_diag_check(P, (uint32_t)(h1 - h0), (unsigned long long *)(c->ws + c->lay.ctl.off + CTL_DIAG),
                                 (double *)(c->ws + c->lay.ctl.off + CTL_DIAG + 8), s));
    }
    return EPIDMC_OK;
}

// The chunks of a run [first, first + n) and the folds of its completed batches, on stream s.
// capture: for a graph (device-driven passes only; no host synchronisation).
static epidmc_status run_range(epidmc_ctx *c, uint64_t first, uint64_t n, hipStream_t s, bool capture, int *nchunks)
{
    const int B = c->batches;
    const int ring = c->lay.ring;
    uint64_t h = first;
    uint64_t next_fold = 0;   // first batch not yet folded
    int chunk = 0;
    while (h < first + n) {
        // a chunk ends at the chunk cap, and never spans more than `ring` batches
        uint64_t h1 = std::min(first + n, h + c->lay.chunk);
        if ((h >> 32) < 0xffffffffull) h1 = std::min(h1, ((h >> 32) + 1) << 32);   // one key per chunk
        const uint64_t b_first = (h - first) * (uint64_t)B / n;
        const uint64_t b_lim = b_first + (uint64_t)ring;   // batches [b_first, b_lim) may be in flight
        if (b_lim < (uint64_t)B) h1 = std::min(h1, batch_start(first, n, B, b_lim));
        REQUIRE(!capture || chunk < MAX_GRAPH_CHUNKS, EPIDMC_E_RANGE, "a captured run holds at most 32 chunks");
        epidmc_status st = run_chunk(c, h, h1, s, capture, chunk);
        if (st != EPIDMC_OK) return st;
        ++chunk;
        // fold the batches that are complete, in batch order (an incomplete batch keeps its slot)
        const uint64_t b_done = (h1 >= first + n) ? (uint64_t)B : (h1 - first) * (uint64_t)B / n;
        while (next_fold < b_done) {
            int slots[MAX_SLOTS];
            double nbs[MAX_SLOTS];
            int k = 0;
            for (; k < MAX_SLOTS && next_fold < b_done; ++k, ++next_fold) {
                slots[k] = (int)(next_fold % (uint64_t)ring);
                nbs[k] = (double)(batch_start(first, n, B, next_fold + 1) - batch_start(first, n, B, next_fold));
            }
            HIPCHK(launch_fold(c->P, slots, nbs, k, s));
        }
        h = h1;
    }
    if (nchunks) *nchunks = chunk;
    return EPIDMC_OK;
}

static void drop_graph(epidmc_ctx *c)
{
    if (c->gx) (void)hipGraphExecDestroy(c->gx);
    if (c->g) (void)hipGraphDestroy(c->g);
    c->gx = nullptr;
    c->g = nullptr;
}

// A run as one graph: captured on the first call for a history range, replayed on later
// calls for the same range (the same histories again), then checked once on the host.
static epidmc_status run_graph(epidmc_ctx *c, uint64_t first, uint64_t n, hipStream_t s)
{
    REQUIRE(c->tally_mode != 2 && !c->diag, EPIDMC_E_ARG, "graph runs need the FP64 or fixed-point tally and diagnostics off");
    if (!c->gx || c->g_first != first || c->g_n != n) {
        drop_graph(c);
        {
            const epidmc_status st = kind_streams(c);
            if (st != EPIDMC_OK) return st;
        }
        if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));   // default priority
        const int passes = c->graph_passes > 0 ? c->graph_passes : (c->last_passes > 0 ? c->last_passes + 2 : 12);
        const int keep = c->graph_passes;
        c->graph_passes = std::min(passes, MAX_DEV_PASSES);
        HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        int nch = 0;
        epidmc_status st = run_range(c, first, n, c->cap, true, &nch);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->cap, &g);
        c->graph_passes = keep;
        if (st != EPIDMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        HIPCHK(ec);
        c->g = g;
        HIPCHK(hipGraphInstantiate(&c->gx, c->g, nullptr, nullptr, 0));
        c->g_first = first;
        c->g_n = n;
        c->g_chunks = nch;
        c->g_passes = passes;
    }
    HIPCHK(hipGraphLaunch(c->gx, s));
    ++c->graph_launches;
    HIPCHK(hipMemcpyAsync(c->host, c->ws + c->lay.ctl.off + CTL_LEFT, (size_t)c->g_chunks * (NQ + 1) * 4,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int ch = 0; ch < c->g_chunks; ++ch)
        for (int k = 0; k < NQ; ++k)
            if (c->host[ch * (NQ + 1) + k]) {
                drop_graph(c);
                return fail(c, EPIDMC_E_OVERFLOW, "a captured run needed more queue passes than the graph holds "
                                                  "(the run's tally is incomplete: reset it, raise the graph's "
                                                  "pass count and run again)");
            }
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_run(epidmc_ctx *c, uint64_t first, uint64_t n, void *stream)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound (call epidmc_bind_workspace after the last set_*)");
    REQUIRE(n >= (uint64_t)c->batches, EPIDMC_E_ARG, "need at least one history per variance batch");
    REQUIRE(first + n > first, EPIDMC_E_RANGE, "history ids must stay below 2^64");
    if (c->n_seg > 1 && c->n_phsp == 0) {
        uint64_t tot = 0;
        for (uint64_t v : c->seg_hist) tot += v;
        REQUIRE(tot > 0, EPIDMC_E_NOT_READY, "the segments hold no histories");
    }
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    c->P.run_first = first;
    c->P.run_n = n;
    c->P.run_batches = c->batches;
    c->P.ring = c->lay.ring;
    epidmc_status st = c->graph ? run_graph(c, first, n, s) : run_range(c, first, n, s, false, nullptr);
    if (st != EPIDMC_OK) return st;
    HIPCHK(hipMemcpyAsync(c->host, c->P.err, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st = check_error_word(c, c->host[0]);
    if (st != EPIDMC_OK) return st;
    c->n_total += (double)n;
    c->b_total += (double)c->batches;
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_read_image(epidmc_ctx *c, double *mean, double *var, void *stream)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    REQUIRE(mean && var, EPIDMC_E_ARG, "null output");
    REQUIRE(c->n_total > 0, EPIDMC_E_NOT_READY, "no histories run");
    HIPCHK(launch_image(c->P, c->n_total, c->b_total, mean, var, (hipStream_t)stream));
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_sigma_bar(epidmc_ctx *c, double thr, void *stream, double *out)
{
    if (!c || !out) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    REQUIRE(c->n_total > 0, EPIDMC_E_NOT_READY, "no histories run");
    REQUIRE(thr >= 0 && thr <= 1, EPIDMC_E_ARG, "threshold fraction in [0,1]");
    hipStream_t s = (hipStream_t)stream;
    double *d = (double *)(c->ws + c->lay.ctl.off + CTL_SIGMA);
    HIPCHK(launch_sigma_bar(c->P, c->n_total, c->b_total, thr, d, s));
    HIPCHK(hipMemcpyAsync(c->host, d, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(out, c->host, 8);
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_run_until(epidmc_ctx *c, double target, double thr, uint64_t first, uint64_t step,
                                          uint64_t max_hist, void *stream, uint64_t *done, double *sb)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(target > 0 && std::isfinite(target), EPIDMC_E_ARG, "target must be > 0");
    REQUIRE(step >= (uint64_t)c->batches && max_hist >= step, EPIDMC_E_ARG, "step >= batches and max >= step");
    uint64_t n = 0;
    double sig = INFINITY;
    while (n + step <= max_hist) {
        epidmc_status st = epidmc_run(c, first + n, step, stream);
        if (st != EPIDMC_OK) return st;
        n += step;
        st = epidmc_sigma_bar(c, thr, stream, &sig);
        if (st != EPIDMC_OK) return st;
        if (sig <= target) break;
    }
    if (done) *done = n;
    if (sb) *sb = sig;
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_reset_tally(epidmc_ctx *c, void *stream)
{
    if (!c) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_zero(c->ws + c->lay.img.off, c->lay.img.bytes, s));
    HIPCHK(launch_zero(c->ws + c->lay.sum.off, c->lay.sum.bytes, s));
    HIPCHK(launch_zero(c->ws + c->lay.sum2.off, c->lay.sum2.bytes, s));
    HIPCHK(launch_zero(c->ws + c->lay.ctl.off, c->lay.ctl.bytes, s));
    HIPCHK(hipStreamSynchronize(s));
    c->n_total = 0;
    c->b_total = 0;
    c->launches = 0;
    c->queue_peak = 0;
    c->last_nrec = 0;
    for (int k = 0; k < NQ; ++k) { c->kernel_ms[k] = 0; c->kernel_launches[k] = 0; }
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_get_counters(epidmc_ctx *c, epidmc_counters *out)
{
    if (!c || !out) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    std::vector<unsigned char> buf(CTL_BYTES);
    HIPCHK(hipMemcpy(buf.data(), c->ws + c->lay.ctl.off, CTL_BYTES, hipMemcpyDeviceToHost));
    unsigned long long st[S_NSTAT];
    std::memcpy(st, buf.data() + CTL_STATS, sizeof st);
    uint32_t err;
    std::memcpy(&err, buf.data() + CTL_ERR, 4);
    unsigned long long mbits;
    double sums[2];
    std::memcpy(&mbits, buf.data() + CTL_DIAG, 8);
    std::memcpy(sums, buf.data() + CTL_DIAG + 8, 16);
    epidmc_counters &o = *out;
    o = epidmc_counters{};
    o.histories = (uint64_t)c->n_total;
    o.n_compton = st[S_COMPTON]; o.n_photo = st[S_PHOTO]; o.n_pair = st[S_PAIR];
    o.n_annih = st[S_ANNIH]; o.n_brems = st[S_BREMS]; o.n_moller = st[S_MOLLER];
    o.woodcock_steps = st[S_WOODCOCK];
    o.epid_photon_steps = st[S_EPID_PH_STEPS];
    o.e_steps_phantom = st[S_ESTEP_P];
    o.e_steps_epid = st[S_ESTEP_E];
    o.photon_epid_entries = st[S_EPID_ENTRIES];
    o.unscattered_at_epid = st[S_UNSCAT];
    o.tally_deposits = st[S_TALLY];
    for (int k = 0; k < 4; ++k) {
        o.queue_items[k] = st[S_ITEMS0 + k];
        o.lane_iters[k] = st[S_LANE0 + k];
        o.wave_iters[k] = st[S_WAVE0 + k];
    }
    o.launches = c->launches;
    o.queue_peak = c->queue_peak;
    o.error_word = err;
    double mx;
    std::memcpy(&mx, &mbits, 8);
    o.max_ledger_resid = mx;
    o.e_in = sums[0];
    o.e_deposited = sums[1];
    o.e_escaped = 0;
    for (int k = 0; k < NQ; ++k) {
        o.kernel_ms[k] = c->kernel_ms[k];
        o.kernel_launches[k] = c->kernel_launches[k];
    }
    return check_error_word(c, err);
}

extern "C" epidmc_status epidmc_radiological_thickness(epidmc_ctx *c, double *dev_out, void *stream)
{
    if (!c || !dev_out) return fail(c, EPIDMC_E_ARG, "null argument");
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    RadArgs A{};
    A.parallel = c->beam.kind == 0;
    A.sx = c->beam.src[0]; A.sy = c->beam.src[1]; A.sz = c->beam.src[2];
    double z = c->front_z;
    for (int l = 0; l < c->scoring; ++l) z += (double)c->layers[l].thickness;
    A.zt = z + 0.5 * (double)c->layers[c->scoring].thickness;
    A.pu = c->pitch_u; A.pv = c->pitch_v;
    A.hx = 0.5 * c->npx_u * A.pu; A.hy = 0.5 * c->npx_v * A.pv;
    A.npx_u = c->npx_u; A.npx_v = c->npx_v;
    A.ox = c->origin[0]; A.oy = c->origin[1]; A.oz = c->origin[2];
    A.dx = c->spacing[0]; A.dy = c->spacing[1]; A.dz = c->spacing[2];
    A.nx = c->nx; A.ny = c->ny; A.nz = c->nz;
    A.vox = c->P.vox;
    A.out = dev_out;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_radthick(A, (hipStream_t)stream));
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_field_size(epidmc_ctx *c, double *s_out)
{
    if (!c || !s_out) return fail(c, EPIDMC_E_ARG, "null argument");
    REQUIRE(c->n_phsp == 0 && c->n_seg > 0, EPIDMC_E_NOT_READY, "no aperture: set_segments first");
    double xmin = INFINITY, xmax = -INFINITY;
    int kmin = -1, kmax = -1;
    for (int g = 0; g < c->n_seg; ++g)
        for (int k = 0; k < c->n_pairs; ++k) {
            const double a = c->ap_a[(size_t)g * c->n_pairs + k], b = c->ap_b[(size_t)g * c->n_pairs + k];
            if (!(b > a)) continue;   // a closed pair
            xmin = std::min(xmin, a);
            xmax = std::max(xmax, b);
            if (kmin < 0 || k < kmin) kmin = k;
            kmax = std::max(kmax, k);
        }
    REQUIRE(kmin >= 0, EPIDMC_E_NOT_READY, "every leaf pair is closed");
    const double A = xmax - xmin, B = (kmax + 1 - kmin) * (double)c->leaf_w;
    *s_out = 2.0 * A * B / (A + B);
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_dose_response(epidmc_ctx *c, const double *dev_image, const double *dev_t, double s,
                                              const double *t_nodes, int nt, const double *s_nodes, int ns,
                                              const double *k, double *dev_out, void *stream)
{
    if (!c || !dev_image || !dev_t || !dev_out || !t_nodes || !s_nodes || !k) return fail(c, EPIDMC_E_ARG, "null argument");
    REQUIRE(nt >= 1 && nt <= RESP_MAX && ns >= 1 && ns <= RESP_MAX, EPIDMC_E_RANGE, "table of 1..64 nodes per axis");
    REQUIRE(std::isfinite(s), EPIDMC_E_RANGE, "field size not finite");
    REQUIRE(c->npx_u > 0 && c->npx_v > 0, EPIDMC_E_NOT_READY, "no EPID image configured");
    for (int i = 0; i < nt; ++i) REQUIRE(std::isfinite(t_nodes[i]) && (i == 0 || t_nodes[i] > t_nodes[i - 1]), EPIDMC_E_RANGE, "t nodes must ascend");
    for (int j = 0; j < ns; ++j) REQUIRE(std::isfinite(s_nodes[j]) && (j == 0 || s_nodes[j] > s_nodes[j - 1]), EPIDMC_E_RANGE, "s nodes must ascend");
    for (int q = 0; q < nt * ns; ++q) REQUIRE(std::isfinite(k[q]), EPIDMC_E_RANGE, "table values must be finite");
    // the two rows bracketing s (clamped), blended: bilinear with s fixed is linear in t on it
    int j = 0;
    double fs = 0.0;
    if (ns > 1 && s > s_nodes[0]) {
        if (s >= s_nodes[ns - 1]) {
            j = ns - 2; fs = 1.0;
        } else {
            while (j + 1 < ns - 1 && s >= s_nodes[j + 1]) ++j;
            fs = (s - s_nodes[j]) / (s_nodes[j + 1] - s_nodes[j]);
        }
    }
    const int j1 = ns > 1 ? j + 1 : j;
    RespArgs A{};
    A.nt = nt;
    for (int i = 0; i < nt; ++i) {
        A.tn[i] = t_nodes[i];
        A.row[i] = (1.0 - fs) * k[j * nt + i] + fs * k[j1 * nt + i];
    }
    A.img = dev_image;
    A.t = dev_t;
    A.out = dev_out;
    A.n = (uint32_t)c->npx_u * (uint32_t)c->npx_v;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_response(A, (hipStream_t)stream));
    return EPIDMC_OK;
}

// clamped bilinear k(t, s) on a rectilinear table (the evaluation k_response performs on
// the device, with s fixed per field)
static double table_bilinear(const double *tn, int nt, const double *sn, int ns, const double *k, double t, double s)
{
    auto bracket = [](const double *x, int n, double v, int &i, double &f) {
        i = 0;
        f = 0.0;
        if (n == 1 || v <= x[0]) return;
        if (v >= x[n - 1]) { i = n - 2; f = 1.0; return; }
        while (i + 1 < n - 1 && v >= x[i + 1]) ++i;
        f = (v - x[i]) / (x[i + 1] - x[i]);
    };
    int i, j;
    double ft, fs;
    bracket(tn, nt, t, i, ft);
    bracket(sn, ns, s, j, fs);
    const int i1 = nt > 1 ? i + 1 : i, j1 = ns > 1 ? j + 1 : j;
    const double r0 = (1.0 - ft) * k[j * nt + i] + ft * k[j * nt + i1];
    const double r1 = (1.0 - ft) * k[j1 * nt + i] + ft * k[j1 * nt + i1];
    return (1.0 - fs) * r0 + fs * r1;
}

extern "C" epidmc_status epidmc_resample_response_table(const double *tn, int nt, const double *sn, int ns, const double *k,
                                                        const double *to, int mt, const double *so, int ms, double *ko)
{
    if (!tn || !sn || !k || !to || !so || !ko) return EPIDMC_E_ARG;
    if (nt < 1 || nt > RESP_MAX || ns < 1 || ns > RESP_MAX || mt < 1 || mt > RESP_MAX || ms < 1 || ms > RESP_MAX)
        return EPIDMC_E_RANGE;
    auto ascending = [](const double *x, int n) {
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(x[i]) || (i > 0 && !(x[i] > x[i - 1]))) return false;
        return true;
    };
    if (!ascending(tn, nt) || !ascending(sn, ns) || !ascending(to, mt) || !ascending(so, ms)) return EPIDMC_E_RANGE;
    for (int q = 0; q < nt * ns; ++q)
        if (!std::isfinite(k[q])) return EPIDMC_E_RANGE;
    for (int j = 0; j < ms; ++j)
        for (int i = 0; i < mt; ++i) ko[j * mt + i] = table_bilinear(tn, nt, sn, ns, k, to[i], so[j]);
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_debug_philox(epidmc_ctx *c, const uint32_t *ctr, uint32_t *out, uint64_t n, void *stream)
{
    if (!c || !ctr || !out || n == 0) return EPIDMC_E_ARG;
    Params P{};
    P.key0 = (uint32_t)c->seed;
    P.key1 = (uint32_t)(c->seed >> 32);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(launch_dbg_philox(P, ctr, out, n, (hipStream_t)stream));
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_debug_sample(epidmc_ctx *c, int kind, double p0, double p1, double p2, float *out,
                                             uint64_t n, void *stream)
{
    if (!c || !out || n == 0 || kind < 0 || kind > 5) return EPIDMC_E_ARG;
    Params P = c->P;
    if (kind == 4) REQUIRE(c->bound, EPIDMC_E_NOT_READY, "source probe needs a bound workspace");
    P.key0 = (uint32_t)c->seed;
    P.key1 = (uint32_t)(c->seed >> 32);
    if (kind == 0 || kind == 5) REQUIRE(p0 > 0 && p0 <= 50, EPIDMC_E_RANGE, "energy in (0, 50]");
    if (kind == 1) REQUIRE(p0 > 2 * WCUT && p0 <= 50, EPIDMC_E_RANGE, "Moller needs T > 0.4 MeV");
    if (kind == 2) REQUIRE(p0 > KCUT && p0 <= 50, EPIDMC_E_RANGE, "bremsstrahlung needs T > 10 keV");
    if (kind == 3) REQUIRE(p0 > 0 && p1 >= 0 && p2 > 0, EPIDMC_E_RANGE, "scattering arguments");
    HIPCHK(hipSetDevice(c->device));
    if (kind == 4) {
        // history ids are integers below 2^53 here; the key takes the high-word mix that
        // run_chunk applies, so the probe draws exactly what k_source draws
        REQUIRE(p0 >= 0 && p0 < 9007199254740992.0 && p0 == std::floor(p0), EPIDMC_E_RANGE,
                "source probe: first history must be a non-negative integer below 2^53");
        const uint64_t h0 = (uint64_t)p0;
        REQUIRE((h0 >> 32) == ((h0 + n - 1) >> 32), EPIDMC_E_RANGE, "source probe range spans a 2^32 boundary");
        const uint32_t hi = (uint32_t)(h0 >> 32);
        P.key0 ^= hi * 0x9E3779B9u;
        P.key1 ^= hi * 0x85EBCA6Bu;
        HIPCHK(launch_dbg_source(P, h0, out, n, (hipStream_t)stream));
        return EPIDMC_OK;
    }
    HIPCHK(launch_dbg_sample(P, kind, (float)p0, (float)p1, (float)p2, out, n, (hipStream_t)stream));
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_debug_queue_capacity(epidmc_ctx *c, int kind, uint32_t per_segment)
{
    if (!c) return EPIDMC_E_ARG;
    // the source writes the phantom photon queue by slot, so only the other kinds can shrink
    REQUIRE(kind >= 1 && kind < NQ, EPIDMC_E_ARG, "kind in [1, 3]");
    REQUIRE(per_segment <= (1u << 24), EPIDMC_E_RANGE, "at most 2^24 particles per segment");
    c->q_override[kind] = per_segment;
    unbind(c);
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_debug_records(epidmc_ctx *c, uint32_t *dev_pix, float *dev_e, uint64_t cap, uint64_t *n,
                                              void *stream)
{
    if (!c || !n || (cap > 0 && (!dev_pix || !dev_e))) return fail(c, EPIDMC_E_ARG, "null argument");
    REQUIRE(c->bound && c->tally_mode == 2, EPIDMC_E_NOT_READY, "records exist in the Kahan tally mode only");
    REQUIRE(c->n_total > 0, EPIDMC_E_NOT_READY, "no histories run");
    *n = c->last_nrec;
    const uint64_t k = std::min<uint64_t>(cap, c->last_nrec);
    if (k == 0) return EPIDMC_OK;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(dev_pix, c->P.rec_pix, k * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(dev_e, c->P.rec_e, k * 4, hipMemcpyDeviceToDevice, s));
    return EPIDMC_OK;
}

extern "C" epidmc_status epidmc_debug_table(epidmc_ctx *c, int kind, int index, const float *E, float *out, uint64_t n,
                                            void *stream)
{
    if (!c || !E || !out || n == 0) return EPIDMC_E_ARG;
    REQUIRE(c->bound, EPIDMC_E_NOT_READY, "workspace not bound");
    REQUIRE(kind >= 0 && kind <= 2 && index >= 0 && index < MAX_PMAT + MAX_LAYERS, EPIDMC_E_ARG, "table kind/index");
    HIPCHK(launch_dbg_table(c->P, kind, index, E, out, n, (hipStream_t)stream));
    return EPIDMC_OK;
}
