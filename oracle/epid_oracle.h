/*
 * epid_oracle.h -- CPU oracle for the EPID transit Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (libepidmc.so and its Python binding) never links, imports or calls it.
 *
 * What it computes: for every EPID pixel, the expected energy deposited in the
 * scoring layer per source history, D_ij, and the variance of its Monte Carlo
 * estimate, by plain FP64 analog Monte Carlo:
 *   - photons: photoelectric, Compton (Klein-Nishina) and pair production, the
 *     three processes the paper models in the patient (Sec. 2.1.2), with cut-offs
 *     of 10 keV for photons and 200 keV for electrons (Sec. 2.1.2);
 *   - electrons: the Class II condensed-history scheme of Sec. 2.1.2 (discrete
 *     hard collisions, continuous slowing down for soft ones), with the step
 *     rules fixed by explicit readings shared with the engine;
 *   - geometry: a voxelised density matrix (Sec. 2.1.2) followed by a stack of
 *     EPID layers (copper build-up, reflector, Gd2O2S phosphor, protective
 *     layers; Sec. 2.1.3) with a 2D pixel grid in the scoring layer.
 * Photons are tracked voxel by voxel (regular tracking, not delta tracking),
 * cross sections are evaluated from their formulas at each energy (no tables),
 * the Klein-Nishina and Moller samplers invert closed-form CDFs numerically, and
 * the variance is accumulated history by history.
 *
 * Units: cm, MeV, g/cm^3.  The library is re-entrant: independent calls on
 * disjoint history ranges may run in parallel threads and their sums are added.
 */
#ifndef EPID_ORACLE_H
#define EPID_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_ELEM   8
#define ORC_MAX_MAT    16
#define ORC_MAX_LAYERS 8

typedef struct {
    int    n_elem;
    int    Z[ORC_MAX_ELEM];
    double A[ORC_MAX_ELEM];   /* g/mol */
    double w[ORC_MAX_ELEM];   /* mass fractions, sum 1 */
    double I_eV;              /* mean excitation energy */
} orc_material;

typedef struct {
    /* physics */
    int      coupled;         /* 0: KERMA (electrons deposit at birth), 1: coupled transport */
    uint32_t proc_mask;       /* bit0 Compton, bit1 photoelectric, bit2 pair;
                                 diagnostic switches: bit3 no hard electron events, bit4 no
                                 multiple scattering */
    double   pcut, ecut;      /* MeV: photon and electron transport cut-offs */
    int      n_mat;
    orc_material mat[ORC_MAX_MAT];
    /* phantom: per-voxel material index and density, x fastest */
    int      nx, ny, nz;
    double   spacing[3];
    double   origin[3];       /* minimum corner */
    const uint8_t *vox_mat;
    const double  *vox_rho;
    /* EPID: contiguous layers starting at front_z, image centred on the z axis */
    int      n_layers;
    int      layer_mat[ORC_MAX_LAYERS];
    double   layer_rho[ORC_MAX_LAYERS];
    double   layer_t[ORC_MAX_LAYERS];
    int      scoring_layer;
    double   front_z;
    int      npx_u, npx_v;    /* u along x (fast index), v along y */
    double   pitch_u, pitch_v;
    /* source */
    int      beam_kind;       /* 0: parallel along +z from the plane z = src[2]; 1: point source at src */
    double   src[3];
    double   iso_z;           /* aperture plane of the point source */
    int      nbins;           /* spectrum: nbins bins, edges[nbins+1], weights[nbins] */
    const double *edges;
    const double *weights;
    int      n_seg, n_pairs;  /* MLC apertures: leaf pair k spans y in [y0+k*w, y0+(k+1)*w) */
    double   leaf_w, y0;
    const double *a, *b;      /* [n_seg][n_pairs] open x interval at the aperture plane */
    const uint64_t *seg_hist; /* [n_seg] histories per segment (global ids are consecutive) */
    uint64_t n_phsp;          /* >0: phase-space list replaces spectrum and aperture */
    const double *phsp;       /* [n_phsp][8]: x y z u v w E type(0 photon, 1 e-, 2 e+) */
    uint64_t seed;
    double   step_floor;      /* a boundary-limited electron step is at least this fraction of the
                                 cell's smallest dimension; the reading is 0 (a step never crosses
                                 a face); other values only serve to measure what a floor does */
} orc_config;

typedef struct {
    uint64_t n_hist;
    uint64_t n_compton, n_photo, n_pair, n_annih, n_brems, n_moller;
    uint64_t e_steps, voxel_visits, photon_epid_entries;
    uint64_t unscattered_at_epid;   /* source photons reaching the EPID front face unscattered */
    uint64_t n_tally_deposits;
    uint64_t n_first_collision;     /* first interactions of source photons in the scoring layer */
    double   e_first_collision;     /* kinetic energy they set in motion */
    double   e_track;               /* total electron path length (cm) */
    double   e_in, e_dep_phantom, e_dep_epid, e_dep_other, e_escaped, e_rest_balance;
    double   max_ledger_resid;      /* max over histories of |ledger residual| / E_in */
} orc_counters;

/* One record of the optional event trace (orc_run_traced), in the order the events happen.
 * Units cm, MeV.  Fields that a kind does not use are zero.
 *   ORC_EV_DEPOSIT  energy E0 left at pos in `region` (0 phantom, 1 EPID, -1 outside both);
 *                   layer = EPID layer or -1; pixel = image index it was tallied to, or -1
 *   ORC_EV_ESTEP    condensed-history step from pos along d0 over aux[0] cm (aux[1] g/cm^2),
 *                   kinetic energy E0 -> E1 (continuous loss), direction after it d1, hinge
 *                   point dc[0]; Ec[0] = radiation length X0 (g/cm^2) of its medium
 *   ORC_EV_COMPTON  photon E0 d0 -> E1 d1 at pos, electron Ec[0] along dc[0]
 *   ORC_EV_PHOTO    photon E0 d0 absorbed at pos, electron Ec[0] along dc[0]
 *   ORC_EV_PAIR     photon E0 d0 at pos -> electron Ec[0] dc[0], positron Ec[1] dc[1]
 *   ORC_EV_ANNIH    positron at rest at pos -> photons Ec[0] dc[0], Ec[1] dc[1]
 *   ORC_EV_MOLLER   electron E0 d0 -> E1 d1 at pos, delta ray Ec[0] dc[0]
 *   ORC_EV_BREMS    electron E0 d0 -> E1 d1 at pos, photon Ec[0] dc[0]
 *   ORC_EV_NULL     a sampled hard-event site rejected as fictitious at pos, energy E0 */
enum { ORC_EV_DEPOSIT = 0, ORC_EV_ESTEP, ORC_EV_COMPTON, ORC_EV_PHOTO, ORC_EV_PAIR, ORC_EV_ANNIH,
       ORC_EV_MOLLER, ORC_EV_BREMS, ORC_EV_NULL };

typedef struct {
    uint64_t hist;
    int32_t  kind, region, layer, pixel;
    double   pos[3];
    double   E0, E1;
    double   d0[3], d1[3];
    double   Ec[2];
    double   dc[2][3];
    double   aux[2];
} orc_event;

/* Return codes */
#define ORC_OK        0
#define ORC_E_ARG    -1
#define ORC_E_LOOP   -2

/* Transport histories [first, first+count).  sum[p] += e_h, sum2[p] += e_h^2 per history
 * for every pixel p = v*npx_u + u (caller zeroes the arrays).  cnt is accumulated into. */
int orc_run(const orc_config *cfg, uint64_t first, uint64_t count,
            double *sum, double *sum2, orc_counters *cnt);

/* orc_run that also records every event into ev[0 .. cap) (see orc_event) and returns the
 * number recorded in *n_ev; events beyond cap are counted in *n_ev but not stored. */
int orc_run_traced(const orc_config *cfg, uint64_t first, uint64_t count,
                   double *sum, double *sum2, orc_counters *cnt, orc_event *ev, uint64_t cap, uint64_t *n_ev);

/* source particle of history h: x y z u v w E type */
int orc_source(const orc_config *cfg, uint64_t h, double out[8]);

/* HU -> (material, density): piecewise-linear density curve (n_pts points, hu ascending,
 * clamped outside) and material ranges: material mat_of[r] for HU < hu_upper[r], first match,
 * the last range catching everything else. */
int orc_map_hu(const int16_t *hu, uint64_t n, int n_pts, const double *curve_hu, const double *curve_rho,
               int n_ranges, const double *hu_upper, const int *mat_of, uint8_t *out_mat, double *out_rho);

/* ---- physics entry points exposed for pinning tests ---- */
double orc_sigma_kn(double E);                       /* cm^2 per electron, closed form */
void   orc_photon_mu(const orc_material *m, double E, double out[4]); /* cm^2/g: total, Compton, photo, pair */
double orc_kn_sample(double E, double xi);            /* epsilon = E'/E by inverse CDF */
double orc_kn_cdf(double E, double eps);              /* normalised CDF of epsilon */
double orc_lcol(const orc_material *m, double T, int restricted, double wcut); /* MeV cm^2/g */
double orc_lres(const orc_material *m, double T, double wcut, double kcut);   /* restricted total */
double orc_sigma_moller(const orc_material *m, double T, double wcut);      /* cm^2/g */
double orc_sigma_brems(const orc_material *m, double T, double kcut);       /* cm^2/g */
double orc_moller_sample(double T, double wcut, double xi);                 /* W (MeV) */
double orc_srad(const orc_material *m, double T);                           /* radiative stopping power */
double orc_brems_sample(double T, double kcut, double xi);                  /* photon energy k (MeV) */
double orc_sigma_hard_max(const orc_material *m, double T0, double wcut, double kcut); /* cm^2/g */
double orc_range_diff(const orc_material *m, double T_lo, double T_hi, double wcut, double kcut); /* g/cm^2 */
double orc_range_inverse(const orc_material *m, double T0, double dR, double wcut, double kcut);
double orc_x0(const orc_material *m);                 /* radiation length, g/cm^2 */
double orc_highland(double T, double x_gcm2, double X0);
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- inputs of the EPID dose-response correction (Sec. 2.2, Sec. 3.1) ---- */
/* Radiological thickness t of the phantom along each pixel's ray, in cm of unit density:
 * the line integral of the voxel density divided by 1 g/cm^3 (Sec. 2.2, item 1).  A
 * point source's ray runs from the source to the pixel centre on the mid-plane of the
 * scoring layer; a parallel beam's runs along +z through the pixel centre.  out[v*npx_u+u].
 * Siddon's method in FP64: every crossing of the ray with a voxel plane inside the box,
 * merged in order; each piece between two crossings contributes its length times the
 * density of the voxel that holds its midpoint. */
int    orc_radiological_thickness(const orc_config *cfg, double *out);
/* the equivalent square (cm) of the bounding rectangle of the open aperture over all
 * segments, at the aperture plane (Sec. 2.2, item 2; Eq. 1 read as 4A/P: s = 2ab/(a+b)) */
double orc_equivalent_square(const orc_config *cfg);
/* k(t,s) by bilinear interpolation on a rectilinear table: t_nodes[nt] and s_nodes[ns]
 * ascending, k[j*nt + i] the factor at (t_i, s_j); outside the table, t and s are clamped to
 * its edges (Eq. 2, Table 1) */
double orc_response_factor(const double *t_nodes, int nt, const double *s_nodes, int ns, const double *k,
                           double t, double s);

#ifdef __cplusplus
}
#endif
#endif
