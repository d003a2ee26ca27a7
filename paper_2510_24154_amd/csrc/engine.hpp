// engine.hpp -- structures shared by the host orchestrator and the gfx950 kernels.
//
// Everything a transport kernel needs travels in one Params struct passed by value:
// device pointers into the caller's workspace, geometry in each region's local
// frame, table grids, the batch layout of the current chunk, and the seed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epidmc {

constexpr int NB_PH = 1024;        // photon table nodes, log-spaced from the photon cut-off
constexpr int NB_EL = 512;         // electron table nodes, log-spaced from half the electron cut-off
constexpr int MAX_PMAT = 4;        // phantom materials (2 bits of the packed voxel word are spare)
constexpr int MAX_LAYERS = 6;
constexpr int MAX_SLOTS = 128;     // variance batches per chunk
constexpr int WG = 256;            // threads per workgroup of the transport kernels
constexpr int WIN = 128;           // queue items a wave claims per atomic
constexpr int SBUF = 64;           // particles a wave stages in LDS per queue kind before one bulk append
constexpr int SBUF_E = 16;         // the same for the electron kernels, whose appends are rarer
constexpr int NSEG = 64;           // segments per queue, each with its own fill counter and consume head
constexpr int CSTRIDE = 32;        // u32 words from one segment counter to the next (one 128-byte line each)
constexpr int ITEMS_PER_LANE = 2;  // a pass launches enough waves for about this many items per lane:
                                   // a wave lives as long as its slowest particle, so thinner waves waste
                                   // lanes, while more items per lane lengthen a small pass, which lasts
                                   // as long as one lane's chain of particles (of 8, 4, 2 and 1, 2 is the
                                   // fastest on short runs and long ones)

// queue kinds: photons / electrons (both signs) x phantom / EPID
enum QKind { QGP = 0, QEP = 1, QGE = 2, QEE = 3, NQ = 4 };

// particle flag bits
constexpr uint32_t F_TYPE = 3u;          // 0 photon, 1 electron, 2 positron
constexpr uint32_t F_UNSCAT = 4u;        // source photon not yet interacted
constexpr uint32_t F_LAYER_SHIFT = 3;    // EPID layer of a photon (3 bits)
constexpr uint32_t F_LAYER_MASK = 7u << F_LAYER_SHIFT;
constexpr uint32_t F_SLOT_SHIFT = 8;     // variance batch slot (8 bits)

// device error word bits
constexpr uint32_t ERR_QUEUE = 1u, ERR_STEPS = 2u, ERR_NAN = 4u, ERR_FIXED = 8u, ERR_SAMPLE = 16u;
constexpr int MAX_KN_ROUNDS = 1000;  // Klein-Nishina draws of one pending sample (acceptance is at least 1/2 per trial)

// model constants of the physics readings (shared meaning with the documentation;
// the numbers are typed here once for the engine)
constexpr double MEC2 = 0.51099895;          // MeV, CODATA 2018
constexpr double RE_CM = 2.8179403262e-13;   // cm
constexpr double NAVO = 6.02214076e23;
constexpr double ALPHA_FS = 1.0 / 137.035999084;
constexpr double C_PE = 2.89e-32;            // photoelectric sigma = C_PE Z^4 / E^3 per atom
constexpr double BREM_K = 800.0;             // S_rad/S_col = Z_eff T / 800 MeV
constexpr double WCUT = 0.200;               // hard Moller threshold, MeV
constexpr double KCUT = 0.010;               // hard bremsstrahlung threshold, MeV
constexpr float NUDGE = 1.0e-5f;             // cm past a boundary for boundary-limited steps
constexpr float DE_FRAC = 0.9f;              // a step keeps at least 90% of its start energy
constexpr int MAX_E_STEPS = 100000;          // per electron and launch; more is an error

// A queued particle is three 16-byte words kept in three arrays of `cap` words
// (a: x y z u, b: v w E hist, c: plo phi draw flags): a lane moves a particle with three
// 128-bit accesses, and a queue costs a kernel three base pointers.
struct Queue {
    uint4 *a, *b, *c;
};

struct Params {
    // queues of this pass: `in` is consumed, `out` is appended to (the host swaps the two
    // buffer sets between passes, so kernels never index them at run time)
    // A queue is NSEG segments of segcap particles; segment s holds items [s segcap, (s+1) segcap).
    // Its fill counter and consume head sit on their own cache lines ([kind][s] x CSTRIDE), so
    // the appends and claims of different waves spread over many addresses instead of
    // serialising on one.
    Queue in[NQ], out[NQ];
    uint32_t segcap[NQ];
    uint32_t *cnt;             // [0, NQ): particles per queue after a pass (summed segments); [3 NQ]: record count
    uint32_t *cnt_in, *cnt_out, *heads;   // segment fill counters being consumed / appended to, consume heads
    uint32_t *err;             // error word
    unsigned long long *stats; // work counters (see Stat)

    // phantom, local frame: box [0,L) with the minimum corner at the origin
    int nx, ny, nz;
    float dx, dy, dz, idx, idy, idz, Lx, Ly, Lz;
    float ox, oy, oz;           // global position of the local origin
    float chord;                // longer than any straight path inside the box
    double ddx, ddy, ddz;       // voxel spacing in FP64 (electron positions are FP64)
    double iddx, iddy, iddz;    // and its inverse
    const uint32_t *vox;        // packed density (bits 31..2) | material (bits 1..0)

    // EPID, local frame: x, y global, z from the front face
    int nl, scoring;
    float zl[MAX_LAYERS + 1];
    float lrho[MAX_LAYERS];
    float front_z, hx, hy;      // front face (global z), lateral half extents
    float zback;                // back face of the last layer (local z)
    int npx_u, npx_v;
    float pitch_u, pitch_v, ipu, ipv, s_pix;
    float ph_to_epid_z;         // front_z - oz: the EPID plane in phantom-local z

    // tables in global memory (the electron kernels copy theirs to LDS; the photon kernels
    // read them through the caches)
    const float *ph_tab;        // [MAX_PMAT + MAX_LAYERS][3][NB_PH]: mu/rho, f_compton, f_compton+photo
    const float *ph_maj;        // [NB_PH] phantom majorant, 1/cm
    const float4 *ph_mu4;       // [NB_PH] mu/rho of the four phantom material slots (0 when unused)
    const float2 *ph_fr;        // [MAX_PMAT][NB_PH] f_compton, f_compton+photo
    float rmaj[MAX_PMAT];       // largest density of each phantom slot x (1 + 1e-5)
    const float *el_tab;        // [MAX_PMAT + MAX_LAYERS][3][NB_EL]: range, sigma_hard, f_moller
    float ph_lnE0, ph_idl;      // photon grid: ln E0 and 1/d(lnE)
    float el_lnT0, el_idl;      // electron grid
    float el_x0[MAX_PMAT + MAX_LAYERS];   // radiation length, g/cm^2
    int nmat_ph;                // phantom materials in use

    // physics
    int coupled;
    uint32_t mask;
    float pcut, ecut;

    // source
    int beam_kind;
    float src[3];               // global
    float iso_z;
    int nbins;
    const float *sp_lo, *sp_hi, *sp_prob;   // [nbins]
    const int *sp_alias;
    int n_seg, n_pairs;
    float leaf_w, y0;
    const float *ap_a, *ap_b, *ap_prob;     // [n_seg][n_pairs]
    const int *ap_alias;
    const unsigned long long *seg_end;      // [n_seg] cumulative history counts
    const float *phsp;                      // [n_phsp][8] or null
    unsigned long long n_phsp;

    // chunk being transported
    unsigned long long h0, h1;  // history ids [h0, h1)
    unsigned long long run_first, run_n;
    int run_batches, ring;      // batch of history h = (h-run_first)*run_batches/run_n; slot = batch % ring
    // device-driven passes: the kinds are launched at their resident grid size whatever their
    // queues hold, and each block first compares its index with the blocks the pass-start
    // kernel's total calls for (about ipl items per lane); 0: the host sized the grid
    int gated;
    int ipl;                    // items per lane the grids are sized for

    // tally
    int tally_mode;
    uint32_t npix;
    void *img;                  // [MAX_SLOTS][npix] doubles or int64
    uint32_t *rec_pix;          // Kahan mode deposit records
    float *rec_e;
    uint32_t rec_cap;
    double *sum, *sum2;         // [npix] folded sums

    // diagnostics
    int diag;
    double *led;                // [h1-h0] per-history ledger
    double *ein;                // [h1-h0] per-history incident energy

    uint32_t key0, key1;
};

// arguments of the radiological-thickness kernel (global frame, cm)
struct RadArgs {
    double sx, sy, sz;      // point source
    double zt;              // plane of the pixel centres: the scoring layer's mid-plane
    int parallel;           // 1: rays along +z through the pixel centres
    double hx, hy, pu, pv;  // image half extents and pitches
    int npx_u, npx_v;
    double ox, oy, oz;      // phantom minimum corner
    double dx, dy, dz;      // voxel spacing
    int nx, ny, nz;
    const uint32_t *vox;    // packed voxels (density bits | material slot)
    double *out;            // [npx_v][npx_u] cm
};

// arguments of the dose-response kernel: the k table at the field's s, as a function of t
constexpr int RESP_MAX = 64;
struct RespArgs {
    int nt;
    double tn[RESP_MAX];    // thickness nodes, ascending
    double row[RESP_MAX];   // k(t_i, s)
    const double *img, *t;
    double *out;
    uint32_t n;
};

enum Stat {
    S_COMPTON = 0, S_PHOTO, S_PAIR, S_ANNIH, S_BREMS, S_MOLLER,
    S_WOODCOCK, S_EPID_PH_STEPS, S_ESTEP_P, S_ESTEP_E, S_EPID_ENTRIES, S_UNSCAT,
    S_TALLY, S_ITEMS0, S_ITEMS1, S_ITEMS2, S_ITEMS3, S_LANE0, S_LANE1, S_LANE2, S_LANE3,
    S_WAVE0, S_WAVE1, S_WAVE2, S_WAVE3, S_NSTAT
};

// diagnostic reduction results live after the stats: max residual (ordered bits), e_in,
// e_dep, e_esc as doubles
constexpr int DIAG_WORDS = 4;

}  // namespace epidmc
