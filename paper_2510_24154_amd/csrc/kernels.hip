// kernels.hip -- gfx950 kernels of the EPID transit Monte Carlo engine.
//
// Transport runs as a loop of queue passes.  Each pass launches one persistent kernel
// per non-empty queue (photons / electrons x phantom / EPID); a wave keeps its 64 lanes
// busy by refilling idle lanes from its queue, advances every lane by one step per loop
// iteration, and appends secondaries and region changes to next-pass queues with one
// atomic per wave.  The electron kernels stage their cross-section tables in LDS once per
// workgroup; the photon kernels read theirs through the caches, where they stay resident
// (in LDS they cost the Woodcock kernel resident waves and made it slower).
//
// Physics per step (the paper's physics class, Sec. 2.1.2; where the paper leaves a model
// open, the engine and the CPU oracle implement the same explicit reading):
//   photons in the phantom: Woodcock delta tracking against a per-energy majorant;
//   photons in the EPID: exact slab-by-slab tracking (Sec. 2.1.3);
//   interactions: Compton (Klein-Nishina, Butcher-Messel composition-rejection),
//     photoelectric absorption, pair production;
//   electrons: Class II condensed history -- steps limited by the sampled distance to a
//     hard event, a 10% energy-loss cap, the cell boundary and half a pixel in the
//     scoring layer; CSDA loss through the restricted range table; random-hinge
//     Gaussian multiple scattering; hard Moller and bremsstrahlung events.
#include "device.hpp"

namespace epidmc {

#define MEC2F 0.51099895f
#define TWO_PI_F 6.28318530717958647692f

struct Local {   // per-lane work counters
    unsigned compton, photo, pair, annih, brems, moller, steps, entries, unscat, tally, items;
};

__device__ __forceinline__ void zero(Local &L) { L = Local{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}; }

__device__ __forceinline__ void flush_stats(const Params &P, const Local &L, int step_stat, int q,
                            unsigned long long lane_iters, unsigned long long wave_iters)
{
    __shared__ unsigned long long s[16];
    if (threadIdx.x < 16) s[threadIdx.x] = 0;
    __syncthreads();
    const unsigned v[11] = {L.compton, L.photo, L.pair, L.annih, L.brems, L.moller, L.steps, L.entries,
                            L.unscat, L.tally, L.items};
#pragma unroll
    for (int k = 0; k < 11; ++k)
        if (v[k]) atomicAdd(&s[k], (unsigned long long)v[k]);
    if (lane_id() == 0) {
        atomicAdd(&s[11], lane_iters);
        atomicAdd(&s[12], wave_iters);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int map[11] = {S_COMPTON, S_PHOTO, S_PAIR, S_ANNIH, S_BREMS, S_MOLLER, step_stat,
                             S_EPID_ENTRIES, S_UNSCAT, S_TALLY, S_ITEMS0 + q};
#pragma unroll
        for (int k = 0; k < 11; ++k)
            if (s[k]) atomicAdd(&P.stats[map[k]], s[k]);
        if (s[11]) atomicAdd(&P.stats[S_LANE0 + q], s[11]);
        if (s[12]) atomicAdd(&P.stats[S_WAVE0 + q], s[12]);
    }
}

// A pass launched without a host round trip starts every kind at its resident grid size;
// the pass-start kernel has just written each queue's total, and the blocks beyond those the
// total calls for (about P.ipl items per lane, as the host sizes grids) leave at once.  The
// test is uniform over the block, before any barrier.
__device__ __forceinline__ bool gated_off(const Params &P, int kind)
{
    if (!P.gated) return false;
    const uint32_t n = __builtin_amdgcn_readfirstlane(P.cnt[kind]);
    const uint32_t per = (uint32_t)WG * (uint32_t)P.ipl;
    return blockIdx.x >= (n + per - 1) / per;
}

// ---------------------------------------------------------------------------------
// placement of a particle given in the phantom frame (source particles, particles that
// leave the phantom box): inside the box it stays; otherwise it flies on a straight line
// to the box (if its ray enters it) or to the EPID front face within the image area, or
// it escapes.  Returns 0 phantom, 1 EPID (p converted to the EPID frame), 2 escaped.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int vacuum_phantom_frame(const Params &P, Part &p)
{
    if (in_phantom(P, p.x, p.y, p.z)) return 0;
    const float pos[3] = {p.x, p.y, p.z}, dir[3] = {p.u, p.v, p.w}, L3[3] = {P.Lx, P.Ly, P.Lz};
    float tin = -INFINITY, tout = INFINITY;
    int ain = -1;
    bool hit = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dir[a] != 0.0f) {
            const float inv = 1.0f / dir[a];
            float t1 = (0.0f - pos[a]) * inv, t2 = (L3[a] - pos[a]) * inv;
            if (t1 > t2) { const float t = t1; t1 = t2; t2 = t; }
            if (t1 > tin) { tin = t1; ain = a; }
            tout = fminf(tout, t2);
        } else if (!(pos[a] >= 0.0f && pos[a] < L3[a])) {
            hit = false;
        }
    }
    if (hit && tin > 0.0f && tin < tout) {
        // the entry point, clamped inside the half-open box; the entry face coordinate exact
        float q0 = fminf(fmaxf(fmaf(tin, p.u, p.x), 0.0f), __uint_as_float(__float_as_uint(P.Lx) - 1u));
        float q1 = fminf(fmaxf(fmaf(tin, p.v, p.y), 0.0f), __uint_as_float(__float_as_uint(P.Ly) - 1u));
        float q2 = fminf(fmaxf(fmaf(tin, p.w, p.z), 0.0f), __uint_as_float(__float_as_uint(P.Lz) - 1u));
        if (ain == 0) q0 = p.u > 0.0f ? 0.0f : __uint_as_float(__float_as_uint(P.Lx) - 1u);
        if (ain == 1) q1 = p.v > 0.0f ? 0.0f : __uint_as_float(__float_as_uint(P.Ly) - 1u);
        if (ain == 2) q2 = p.w > 0.0f ? 0.0f : __uint_as_float(__float_as_uint(P.Lz) - 1u);
        p.x = q0; p.y = q1; p.z = q2;
        return 0;
    }
    if (p.w > 0.0f) {
        const float t = (P.ph_to_epid_z - p.z) / p.w;
        const float xg = fmaf(t, p.u, p.x) + P.ox, yg = fmaf(t, p.v, p.y) + P.oy;
        if (xg >= -P.hx && xg < P.hx && yg >= -P.hy && yg < P.hy) {
            p.x = xg; p.y = yg; p.z = 0.0f;
            return 1;
        }
    }
    return 2;
}

// hand a particle (position in the frame of `region`) to its next queue, or let it escape
__device__ __forceinline__ void place(const Params &P, int region, Part &c, Local &L, Stages S = no_stages())
{
    const bool photon = (c.flags & F_TYPE) == 0;
    int r = region;
    if (region == 0) {
        r = vacuum_phantom_frame(P, c);
        if (r == 1 && photon) {
            ++L.entries;
            if (c.flags & F_UNSCAT) ++L.unscat;
        }
    } else {
        if (epid_layer(P, c.x, c.y, c.z) < 0) r = 2;
    }
    if (r == 2) {
        ledger(P, c.hist, (double)c.E);
        return;
    }
    if (r == 1 && photon) {
        const int l = max(epid_layer(P, c.x, c.y, c.z), 0);
        c.flags = (c.flags & ~F_LAYER_MASK) | ((uint32_t)l << F_LAYER_SHIFT);
    }
    const int kind = (r == 0) ? (photon ? QGP : QEP) : (photon ? QGE : QEE);
    // appends are grouped by kind so each call ballots only the lanes of that kind
    append(P, S, QGP, kind == QGP, c);
    append(P, S, QEP, kind == QEP, c);
    append(P, S, QGE, kind == QGE, c);
    append(P, S, QEE, kind == QEE, c);
}

// A photon outside the phantom box whose ray cannot enter it (it has just left the box on a
// straight line, or it is a source photon whose ray misses the box): it reaches the EPID
// front face within the image area, or it escapes.
__device__ __forceinline__ void photon_leaves_phantom(const Params &P, Part &p, Local &L, Stages S)
{
    if (p.w > 0.0f) {
        const float t = (P.ph_to_epid_z - p.z) / p.w;
        const float xg = fmaf(t, p.u, p.x) + P.ox, yg = fmaf(t, p.v, p.y) + P.oy;
        if (xg >= -P.hx && xg < P.hx && yg >= -P.hy && yg < P.hy) {
            p.x = xg; p.y = yg; p.z = 0.0f;
            p.flags &= ~F_LAYER_MASK;   // the front layer
            ++L.entries;
            if (p.flags & F_UNSCAT) ++L.unscat;
            append(P, S, QGE, true, p);
            return;
        }
    }
    ledger(P, p.hist, (double)p.E);
}

// deposit at a point of `region` (phantom: ledger only; EPID: tallied in the scoring layer)
__device__ __forceinline__ void deposit_point(const Params &P, int region, const Part &at, float e, Local &L)
{
    ledger(P, at.hist, (double)e);
    if (region == 1) {
        unsigned n = 0;
        deposit_epid_point(P, at, e, n);
        L.tally += n;
    }
}

// a new photon at the parent's position
__device__ __forceinline__ void emit_photon(const Params &P, int region, Part &parent, float E, float u, float v, float w,
                            Local &L, Stages S = no_stages())
{
    Part c;
    make_child(parent, c, 0u);
    c.x = parent.x; c.y = parent.y; c.z = parent.z;
    c.u = u; c.v = v; c.w = w;
    c.E = E;
    if (E < P.pcut) {
        deposit_point(P, region, c, E, L);
        return;
    }
    place(P, region, c, L, S);
}

// two back-to-back photons of m c^2 from a positron at rest
__device__ __forceinline__ void annihilate(const Params &P, int region, Part &pos, Local &L, Stages S = no_stages())
{
    const float4 r = rnd4(pos, P);
    const float ct = 2.0f * r.x - 1.0f, st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float sp, cp;
    __sincosf(TWO_PI_F * r.y, &sp, &cp);
    ++L.annih;
    ledger(P, pos.hist, -2.0 * (double)MEC2F);
    emit_photon(P, region, pos, MEC2F, st * cp, st * sp, ct, L, S);
    emit_photon(P, region, pos, MEC2F, -st * cp, -st * sp, -ct, L, S);
}

// a new electron (type 1) or positron (type 2) at the parent's position
__device__ __forceinline__ void emit_electron(const Params &P, int region, Part &parent, float T, uint32_t type, float u, float v,
                              float w, Local &L, Stages S = no_stages())
{
    Part c;
    make_child(parent, c, type);
    c.x = parent.x; c.y = parent.y; c.z = parent.z;
    c.u = u; c.v = v; c.w = w;
    c.E = T;
    if (!P.coupled || T < P.ecut) {
        deposit_point(P, region, c, T, L);
        if (type == 2u) annihilate(P, region, c, L, S);
        return;
    }
    place(P, region, c, L, S);
}

// ---------------------------------------------------------------------------------
// samplers
// ---------------------------------------------------------------------------------
// Klein-Nishina eps = E'/E by the Butcher-Messel split of (1/eps + eps) into a 1/eps part
// (eps = eps0^u) and an eps part (eps^2 uniform on [eps0^2, 1]), with the rejection function
// 1 - eps sin^2 / (1 + eps^2).  A trial takes two uniforms: u1 picks the part with
// probability a1 / (a1 + a2) and, rescaled to (0, 1) within it, gives the trial eps; u2 is
// the acceptance variate, and on acceptance u2 / g is uniform on (0, 1) independently of
// eps, which gives the azimuth.
struct KN {
    float k, e0, e02, a1, pa, ipa, iqa;
};

__device__ __forceinline__ KN kn_setup(float E)
{
    KN c;
    c.k = E * (1.0f / MEC2F);
    const float d = fmaf(2.0f, c.k, 1.0f);
    c.e0 = 1.0f / d;
    c.a1 = __logf(d);
    c.e02 = c.e0 * c.e0;
    const float a2 = 0.5f * (1.0f - c.e02);
    c.pa = c.a1 / (c.a1 + a2);
    c.ipa = 1.0f / c.pa;
    c.iqa = 1.0f / (1.0f - c.pa);
    return c;
}

__device__ __forceinline__ bool kn_trial(const KN &c, float u1, float u2, float &eps, float &t, float &phu)
{
    float e = u1 < c.pa ? __expf(-c.a1 * (u1 * c.ipa)) : sqrtf(fmaf(1.0f - c.e02, (u1 - c.pa) * c.iqa, c.e02));
    e = fminf(fmaxf(e, c.e0), 1.0f);
    const float tt = (1.0f - e) / (c.k * e);
    const float g = 1.0f - e * (tt * (2.0f - tt)) / fmaf(e, e, 1.0f);
    if (!(u2 < g)) return false;
    eps = e;
    t = fminf(tt, 2.0f);
    phu = fminf(u2 / g, 0.99999994f);
    return true;
}

// a complete Klein-Nishina sample: trials two per Philox draw until one is accepted
__device__ __forceinline__ float kn_sample(const Params &P, Part &p, float E, float &t_out, float &phi_u)
{
    const KN c = kn_setup(E);
    float eps = 1.0f, t = 0.0f, phu = 0.5f;
    for (int draw = 0; draw < 5000; ++draw) {
        const float4 r = rnd4(p, P);
        if (kn_trial(c, r.x, r.y, eps, t, phu) || kn_trial(c, r.z, r.w, eps, t, phu)) break;
    }
    t_out = t;
    phi_u = phu;
    return eps;
}

// Moller energy transfer W = eps T in [WCUT, T/2]: a 1/eps^2 proposal on [WCUT/T, 1/2] from
// u1, accepted with u2 against the rest of the Moller bracket, which 2 + c1/4 bounds on the
// interval
struct MollerC {
    float ec, c1, c2, bound;
};

__device__ __forceinline__ MollerC moller_setup(float T)
{
    MollerC m;
    m.ec = (float)WCUT / T;
    const float g = T * (1.0f / MEC2F) + 1.0f;
    m.c1 = (g - 1.0f) * (g - 1.0f) / (g * g);
    m.c2 = (2.0f * g - 1.0f) / (g * g);
    m.bound = 2.0f + 0.25f * m.c1;
    return m;
}

__device__ __forceinline__ bool moller_trial(const MollerC &m, float u1, float u2, float &eps)
{
    const float e = m.ec / (1.0f - u1 * (1.0f - 2.0f * m.ec));
    const float x = e / (1.0f - e);
    const float gf = 1.0f + x * x + m.c1 * e * e - m.c2 * x;
    eps = fminf(fmaxf(e, m.ec), 0.5f);
    return u2 * m.bound < gf;
}

// a complete Moller sample (one trial per Philox draw until accepted); also returns the
// azimuth uniform of the accepted trial
__device__ __forceinline__ float moller_sample(const Params &P, Part &p, float T, float &phi_u)
{
    const MollerC m = moller_setup(T);
    float eps = m.ec;
    for (int trial = 0; trial < 10000; ++trial) {
        const float4 r = rnd4(p, P);
        phi_u = r.z;
        if (moller_trial(m, r.x, r.y, eps)) break;
    }
    return eps * T;
}

// bremsstrahlung photon energy from the 1/k spectrum on [KCUT, T]: k = KCUT (T / KCUT)^u
__device__ __forceinline__ float brems_k(float T, float u)
{
    return (float)KCUT * __expf(u * __logf(T * (float)(1.0 / KCUT)));
}

// Highland width (unit charge) for kinetic energy T over x g/cm^2 of radiation length X0
__device__ __forceinline__ float highland(float T, float x, float X0)
{
    if (!(x > 0.0f)) return 0.0f;
    const float E = T + MEC2F;
    const float iE = 1.0f / E;
    const float pc2 = T * (T + 2.0f * MEC2F);
    const float b2 = pc2 * iE * iE;
    const float r = x / X0;
    const float br = fmaxf(0.0f, 1.0f + 0.038f * __logf(r / b2));
    return 13.6f * E / pc2 * sqrtf(r) * br;
}

// ---------------------------------------------------------------------------------
// photon interactions (the photon kernels inline the common Compton and photoelectric paths)
// ---------------------------------------------------------------------------------
// Compton kinematics in place: the photon p turns by (t = 1 - cos theta, azimuth uniform
// phu) and keeps eps E; returns the electron's kinetic energy, with its direction, the one
// that conserves momentum (incident minus scattered photon momentum), in (eu, ev, ew).
__device__ __forceinline__ float compton_kin(const Params &P, Part &p, float eps, float t, float phu, float &eu,
                                             float &ev, float &ew)
{
    const float E = p.E;
    const float ct = 1.0f - t, st = sqrtf(fmaxf(0.0f, t * (2.0f - t)));
    float sp, cp;
    __sincosf(TWO_PI_F * phu, &sp, &cp);
    const float Ep = eps * E, eT = E - Ep;
    if (P.diag) ledger(P, p.hist, (double)E - (double)Ep - (double)eT);
    eu = p.u; ev = p.v; ew = p.w;
    rotate(p.u, p.v, p.w, ct, st, cp, sp);
    const float qx = fmaf(-Ep, p.u, E * eu), qy = fmaf(-Ep, p.v, E * ev), qz = fmaf(-Ep, p.w, E * ew);
    const float q2 = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
    if (q2 > 0.0f) {
        const float iq = rsqrtf(q2);
        eu = qx * iq; ev = qy * iq; ew = qz * iq;
    }
    p.E = Ep;
    return eT;
}

// pair production: the electron takes a uniform share u of E - 2 m c^2, the positron the rest,
// both along the photon
__device__ __forceinline__ void pair_produce(const Params &P, int region, Part &p, float u, Local &L, Stages S)
{
    ++L.pair;
    const float E = p.E;
    const float T = E - 2.0f * MEC2F;
    const float tm = u * T, tp = T - tm;
    if (P.diag) ledger(P, p.hist, (double)E - (double)tm - (double)tp);
    emit_electron(P, region, p, tm, 1u, p.u, p.v, p.w, L, S);
    emit_electron(P, region, p, tp, 2u, p.u, p.v, p.w, L, S);
}

// ---------------------------------------------------------------------------------
// source: one thread per history
// ---------------------------------------------------------------------------------
// The source particle of history h in the global frame, a stand-in for the particles that
// leave the collimators (Sec. 2.1.1): particle h mod n of a phase-space list, or a photon
// whose energy comes from the spectrum's alias table and whose direction aims at a point
// drawn uniformly over the open area of the history's segment (a leaf pair from the
// segment's alias table over open widths, then a point uniform within the pair).  The
// history's random stream starts at draw 0 with particle id 0.
__device__ __forceinline__ void source_particle(const Params &P, unsigned long long h, Part &p, float &gx, float &gy,
                                                float &gz, uint32_t &type)
{
    p.hist = (uint32_t)h;
    p.plo = 0; p.phi = 0; p.draw = 0;
    type = 0;
    if (P.n_phsp) {
        const float *q = P.phsp + 8 * (h % P.n_phsp);
        gx = q[0]; gy = q[1]; gz = q[2];
        p.u = q[3]; p.v = q[4]; p.w = q[5];
        p.E = q[6];
        type = (uint32_t)q[7];
        return;
    }
    const float4 r = rnd4(p, P);
    int i = min((int)(r.x * (float)P.nbins), P.nbins - 1);
    if (r.y >= P.sp_prob[i]) i = P.sp_alias[i];
    p.E = fmaf(r.z, P.sp_hi[i] - P.sp_lo[i], P.sp_lo[i]);
    int s = 0;
    if (P.n_seg > 1) {
        // ids past the field's total deliver it again: the segment of h mod total, with the
        // history's own random stream
        const unsigned long long tot = P.seg_end[P.n_seg - 1];
        const unsigned long long hs = h < tot ? h : h % tot;
        int lo = 0, hi = P.n_seg - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (hs < P.seg_end[mid]) hi = mid; else lo = mid + 1;
        }
        s = lo;
    }
    const float4 r2 = rnd4(p, P);
    const int base = s * P.n_pairs;
    int k = min((int)(r2.x * (float)P.n_pairs), P.n_pairs - 1);
    if (r2.y >= P.ap_prob[base + k]) k = P.ap_alias[base + k];
    const float a = P.ap_a[base + k], b = P.ap_b[base + k];
    const float x = fmaf(r2.z, b - a, a);
    const float y = fmaf((float)k + r2.w, P.leaf_w, P.y0);
    if (P.beam_kind == 0) {
        gx = x; gy = y; gz = P.src[2];
        p.u = 0.0f; p.v = 0.0f; p.w = 1.0f;
    } else {
        const float dx = x - P.src[0], dy = y - P.src[1], dz = P.iso_z - P.src[2];
        const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
        gx = P.src[0]; gy = P.src[1]; gz = P.src[2];
        p.u = dx * inv; p.v = dy * inv; p.w = dz * inv;
    }
}

__global__ __launch_bounds__(WG) void k_source(Params P)
{
    Local L;
    zero(L);
    const unsigned long long h = P.h0 + (unsigned long long)blockIdx.x * WG + threadIdx.x;
    const bool live = h < P.h1;
    if (live) {
        const uint32_t slot = (uint32_t)(((h - P.run_first) * (unsigned long long)P.run_batches / P.run_n) % P.ring);
        Part p;
        float gx = 0, gy = 0, gz = 0;
        uint32_t type = 0;
        source_particle(P, h, p, gx, gy, gz, type);
        p.flags = (slot << F_SLOT_SHIFT) | type | (type == 0 ? F_UNSCAT : 0u);
        if (P.diag) P.ein[h - P.h0] = (double)p.E;
        p.x = gx - P.ox; p.y = gy - P.oy; p.z = gz - P.oz;
        if (!P.n_phsp) {
            // spectrum source: every history is one photon.  It takes slot h - h0 of the photon
            // queue directly (no atomics); one that misses the phantom box is stored where it
            // is and placed by the Woodcock kernel when loaded.
            if (!in_phantom(P, p.x, p.y, p.z)) {
                Part q = p;
                if (vacuum_phantom_frame(P, q) == 0) p = q;   // moved to its entry point
            }
            // item j of the chunk goes to segment j / q at offset j % q, q = ceil(n / NSEG)
            const uint32_t j = (uint32_t)(h - P.h0), q = (uint32_t)((P.h1 - P.h0 + NSEG - 1) / NSEG);
            const uint32_t sg = j / q;
            qstore(P.out[QGP], sg * P.segcap[QGP] + (j - sg * q), p);
        } else if (in_phantom(P, p.x, p.y, p.z)) {
            // a phase-space particle that starts inside the box is in the phantom
            const bool photon = type == 0;
            qappend(P, QGP, photon, p, home_seg());
            qappend(P, QEP, !photon, p, home_seg());
        } else {
            place(P, 0, p, L);
        }
    }
    if (!P.n_phsp && blockIdx.x == 0 && threadIdx.x < NSEG) {
        const uint32_t n = (uint32_t)(P.h1 - P.h0), q = (n + NSEG - 1) / NSEG, s0 = threadIdx.x * q;
        *seg_ctr(P.cnt_out, QGP, threadIdx.x) = s0 < n ? min(q, n - s0) : 0u;
    }
    // counters of direct hits on the EPID
    if (L.entries) atomicAdd(&P.stats[S_EPID_ENTRIES], (unsigned long long)L.entries);
    if (L.unscat) atomicAdd(&P.stats[S_UNSCAT], (unsigned long long)L.unscat);
}

// ---------------------------------------------------------------------------------
// photons in the phantom: Woodcock tracking
// ---------------------------------------------------------------------------------
// Six waves per SIMD (the most the LDS staging allows: six workgroups per CU): the kernel
// is VALU-bound on divergent code and its voxel gathers miss L2 about half the time, so the
// extra wave hides latency.  It costs one spilled register.
__global__ __launch_bounds__(WG, 6) void k_photon_phantom(Params P)
{
    if (gated_off(P, QGP)) return;
    // dynamic LDS: per wave two staging buffers (electrons for the phantom queue, photons
    // for the EPID queue).  The packed tables (16 KB of mu/rho, 32 KB of process fractions)
    // stay in global memory, where they live in L2.
    extern __shared__ __align__(16) float lds[];
    Stages S;
    stage_carve(S, (uint32_t *)lds + (size_t)wave_id() * 2 * stage_words(SBUF), (1u << QEP) | (1u << QGE), SBUF);
    __syncthreads();

    Win win = win_start();
    bool active = false;
    bool kn = false;   // a Compton collision whose Klein-Nishina sample is still pending
    int kn_rounds = 0; // draws spent on it
    Part p;
    Local L;
    zero(L);
    unsigned long long lane_iters = 0, wave_iters = 0;
    for (;;) {
        stage_flush_all(P, S, SBUF / 2);
        const bool was = active;
        refill(P, QGP, win, active, p);
        const unsigned long long act = __ballot(active);
        if (act == 0) break;
        lane_iters += __popcll(act);
        wave_iters += 64;
        // Control flow merges before every shared piece (the exit to the EPID, the Klein-
        // Nishina trial, the electron emission), so that each is compiled once: a wave runs
        // every piece that any of its lanes needs on every iteration.
        bool leave = false;   // outside the box on a ray that cannot enter it: EPID or escape
        if (active && !was) {
            ++L.items;
            kn = false;
            leave = !in_phantom(P, p.x, p.y, p.z);   // a source photon whose ray misses the box
        }
        if (active && !leave) {
            // mu/rho of the four phantom slots at p.E.  Recomputed on every iteration: some lane
            // of the wave takes a new energy on nearly every iteration, so a per-lane cache would
            // save no wave instructions, and its registers are worth the sixth wave.
            const Node nd = node_of(__logf(p.E), P.ph_lnE0, P.ph_idl, NB_PH);
            const float4 a = P.ph_mu4[nd.i], b = P.ph_mu4[nd.i + 1];
            const float4 mu = make_float4(fmaf(nd.f, b.x - a.x, a.x), fmaf(nd.f, b.y - a.y, a.y),
                                          fmaf(nd.f, b.z - a.z, a.z), fmaf(nd.f, b.w - a.w, a.w));
            // the majorant: each slot's largest density times its mu/rho, so that it bounds
            // rho mu/rho of every voxel at this energy exactly as interpolated here
            const float mubar =
                fmaxf(fmaxf(P.rmaj[0] * mu.x, P.rmaj[1] * mu.y), fmaxf(P.rmaj[2] * mu.z, P.rmaj[3] * mu.w));
            const float imubar = 1.0f / mubar;
            // One Philox draw per lane and iteration, so that every lane of the wave spends its
            // random-number work together: a flight uses it for the distance, the real/virtual
            // test, the process and the first Klein-Nishina trial; a pending Compton sample
            // uses it for two further trials.
            const float4 r = rnd4(p, P);
            bool trial = kn;       // a Klein-Nishina trial this iteration, from (u1, u2)
            bool absorb = false;   // photoelectric absorption: the electron takes E along the photon
            float u1 = r.x, u2 = r.y;
            if (!kn) {
                // a flight longer than the box chord leaves the box either way (and an empty
                // phantom, mubar = 0, must not produce an infinite step)
                const float s = fminf(-__logf(r.x) * imubar, P.chord);
                p.x = fmaf(s, p.u, p.x);
                p.y = fmaf(s, p.v, p.y);
                p.z = fmaf(s, p.w, p.z);
                ++L.steps;
                leave = !in_phantom(P, p.x, p.y, p.z);   // left the box on a straight line
                if (!leave) {
                    const int ix = min((int)(p.x * P.idx), P.nx - 1), iy = min((int)(p.y * P.idy), P.ny - 1),
                              iz = min((int)(p.z * P.idz), P.nz - 1);
                    const uint32_t word =
                        P.vox[((uint32_t)iz * (uint32_t)P.ny + (uint32_t)iy) * (uint32_t)P.nx + (uint32_t)ix];
                    const float rho = __uint_as_float(word & ~3u);
                    const int m = (int)(word & 3u);
                    const float mum = m == 0 ? mu.x : m == 1 ? mu.y : m == 2 ? mu.z : mu.w;
                    if (r.y * mubar < rho * mum) {
                        // a real collision: r.z picks the process, and within Compton, rescaled
                        // to (0, 1), it is the first trial's part-and-eps uniform
                        const float2 fa = P.ph_fr[m * NB_PH + nd.i], fb = P.ph_fr[m * NB_PH + nd.i + 1];
                        const float fc = fmaf(nd.f, fb.x - fa.x, fa.x);
                        p.flags &= ~F_UNSCAT;
                        if (r.z < fc) {
                            ++L.compton;
                            trial = true;
                            u1 = fminf(r.z / fc, 0.99999994f);
                            u2 = r.w;
                        } else if (r.z < fmaf(nd.f, fb.y - fa.y, fa.y)) {
                            ++L.photo;
                            absorb = true;
                        } else {
                            pair_produce(P, 0, p, r.w, L, S);   // rare: kept out of the merged path
                            active = false;
                        }
                    }
                }
            }
            float eps = 1.0f, t = 0.0f, phu = 0.0f;
            bool scatter = false;
            if (trial) {
                const KN c = kn_setup(p.E);
#pragma unroll 1
                for (int k = 0; k < 2; ++k) {
                    scatter = kn_trial(c, u1, u2, eps, t, phu);
                    if (scatter || !kn) break;
                    u1 = r.z;   // a pending sample gets a second trial from the same draw
                    u2 = r.w;
                }
                kn_rounds = kn ? kn_rounds + 1 : 0;
                kn = !scatter;
                if (kn && kn_rounds > MAX_KN_ROUNDS) {
                    // unreachable with a sound generator; ends the lane so the wave drains
                    atomicOr(P.err, ERR_SAMPLE);
                    ledger(P, p.hist, (double)p.E);
                    kn = false;
                    active = false;
                }
            }
            if (scatter || absorb) {
                // one electron set in motion at p: after a Compton scatter it carries the
                // momentum the photon lost, after absorption the photon's energy and direction
                const float E = p.E;
                float eT = E, eu = p.u, ev = p.v, ew = p.w;
                active = false;
                if (scatter) {
                    eT = compton_kin(P, p, eps, t, phu, eu, ev, ew);
                    active = p.E >= P.pcut;
                    if (!active) ledger(P, p.hist, (double)p.E);
                }
                Part c;
                make_child(p, c, 1u);
                c.x = p.x; c.y = p.y; c.z = p.z;
                c.u = eu; c.v = ev; c.w = ew;
                c.E = eT;
                if (!P.coupled || eT < P.ecut) ledger(P, c.hist, (double)eT);
                else append(P, S, QEP, true, c);
            }
        }
        if (leave) {
            photon_leaves_phantom(P, p, L, S);
            active = false;
        }
    }
    stage_flush_all(P, S, 1);
    flush_stats(P, L, S_WOODCOCK, QGP, lane_iters, wave_iters);
}


// ---------------------------------------------------------------------------------
// photons in the EPID: exact tracking across the slabs
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_photon_epid(Params P)
{
    if (gated_off(P, QGE)) return;
    // dynamic LDS: per wave one staging buffer for the electrons set in motion in the EPID.
    // The layer tables (48 KB for four layers) are read from global memory, where they stay
    // in the caches: in LDS they made a workgroup too large to fit beside the phantom
    // electron kernel, which runs in the same passes, and this kernel then ran on the few
    // CUs that kernel left free.
    extern __shared__ __align__(16) float lds[];
    __shared__ float s_zl[MAX_LAYERS + 1], s_rho[MAX_LAYERS];
    const float *ltab = P.ph_tab + MAX_PMAT * 3 * NB_PH;
    Stages S;
    stage_carve(S, (uint32_t *)lds + wave_id() * stage_words(SBUF), 1u << QEE, SBUF);
    if (threadIdx.x <= MAX_LAYERS) s_zl[threadIdx.x] = P.zl[threadIdx.x];
    if (threadIdx.x < MAX_LAYERS) s_rho[threadIdx.x] = P.lrho[threadIdx.x];
    __syncthreads();

    Win win = win_start();
    bool active = false;
    bool kn = false;     // a Compton collision whose Klein-Nishina sample is still pending
    int kn_rounds = 0;
    Part p;
    Local L;
    zero(L);
    unsigned long long lane_iters = 0, wave_iters = 0;
    for (;;) {
        stage_flush_all(P, S, SBUF / 2);
        const bool was = active;
        refill(P, QGE, win, active, p);
        const unsigned long long act = __ballot(active);
        if (act == 0) break;
        lane_iters += __popcll(act);
        wave_iters += 64;
        if (active && !was) {
            ++L.items;
            kn = false;
        }
        if (!active) continue;
        // one Philox draw per lane and iteration (as in the Woodcock kernel): a flight uses it
        // for the distance, the process and the first Klein-Nishina trial; a pending Compton
        // sample uses it for two further trials
        const float4 r = rnd4(p, P);
        bool trial = kn, absorb = false;
        float u1 = r.x, u2 = r.y;
        if (!kn) {
            const int l = (int)((p.flags & F_LAYER_MASK) >> F_LAYER_SHIFT);
            const float *tab = ltab + l * 3 * NB_PH;
            const Node nd = node_of(__logf(p.E), P.ph_lnE0, P.ph_idl, NB_PH);
            const float mu = s_rho[l] * lerp_tab(tab, nd);
            // distance to the slab planes and to the lateral faces
            float tz = INFINITY;
            int dl = 0;
            if (p.w > 0.0f) { tz = (s_zl[l + 1] - p.z) / p.w; dl = 1; }
            else if (p.w < 0.0f) { tz = (s_zl[l] - p.z) / p.w; dl = -1; }
            float tl = INFINITY;
            if (p.u > 0.0f) tl = fminf(tl, (P.hx - p.x) / p.u);
            else if (p.u < 0.0f) tl = fminf(tl, (-P.hx - p.x) / p.u);
            if (p.v > 0.0f) tl = fminf(tl, (P.hy - p.y) / p.v);
            else if (p.v < 0.0f) tl = fminf(tl, (-P.hy - p.y) / p.v);
            tz = fmaxf(tz, 0.0f);
            tl = fmaxf(tl, 0.0f);
            const float s = -__logf(r.x) / mu;
            ++L.steps;
            if (s < fminf(tz, tl)) {
                p.x = fmaf(s, p.u, p.x);
                p.y = fmaf(s, p.v, p.y);
                p.z = fmaf(s, p.w, p.z);
                // a collision: r.y picks the process and, rescaled within Compton, is the first
                // trial's part-and-eps uniform
                const float fc = lerp_tab(tab + NB_PH, nd);
                p.flags &= ~F_UNSCAT;
                if (r.y < fc) {
                    ++L.compton;
                    trial = true;
                    u1 = fminf(r.y / fc, 0.99999994f);
                    u2 = r.z;
                } else if (r.y < lerp_tab(tab + 2 * NB_PH, nd)) {
                    ++L.photo;
                    absorb = true;
                } else {
                    pair_produce(P, 1, p, r.z, L, S);   // rare: kept out of the merged path
                    active = false;
                }
            } else if (tl <= tz) {   // leaves through a lateral face
                ledger(P, p.hist, (double)p.E);
                active = false;
            } else {
                p.x = fmaf(tz, p.u, p.x);
                p.y = fmaf(tz, p.v, p.y);
                const int nlay = l + dl;
                if (nlay < 0 || nlay >= P.nl) {
                    ledger(P, p.hist, (double)p.E);
                    active = false;
                } else {
                    p.z = dl > 0 ? s_zl[l + 1] : s_zl[l];
                    p.flags = (p.flags & ~F_LAYER_MASK) | ((uint32_t)nlay << F_LAYER_SHIFT);
                }
            }
        }
        float eps = 1.0f, t = 0.0f, phu = 0.0f;
        bool scatter = false;
        if (trial) {
            const KN c = kn_setup(p.E);
#pragma unroll 1
            for (int k = 0; k < 2; ++k) {
                scatter = kn_trial(c, u1, u2, eps, t, phu);
                if (scatter || !kn) break;
                u1 = r.z;   // a pending sample gets a second trial from the same draw
                u2 = r.w;
            }
            kn_rounds = kn ? kn_rounds + 1 : 0;
            kn = !scatter;
            if (kn && kn_rounds > MAX_KN_ROUNDS) {
                atomicOr(P.err, ERR_SAMPLE);   // unreachable with a sound generator
                ledger(P, p.hist, (double)p.E);
                kn = false;
                active = false;
            }
        }
        if (scatter || absorb) {
            // one electron set in motion at p, inside the EPID layer the photon is in
            float eT = p.E, eu = p.u, ev = p.v, ew = p.w;
            active = false;
            if (scatter) {
                eT = compton_kin(P, p, eps, t, phu, eu, ev, ew);
                active = p.E >= P.pcut;
                if (!active) deposit_point(P, 1, p, p.E, L);
            }
            Part c;
            make_child(p, c, 1u);
            c.x = p.x; c.y = p.y; c.z = p.z;
            c.u = eu; c.v = ev; c.w = ew;
            c.E = eT;
            if (!P.coupled || eT < P.ecut) deposit_point(P, 1, c, eT, L);
            else append(P, S, QEE, true, c);
        }
    }
    stage_flush_all(P, S, 1);
    flush_stats(P, L, S_EPID_PH_STEPS, QGE, lane_iters, wave_iters);
}

// ---------------------------------------------------------------------------------
// electrons and positrons: Class II condensed history, one step per loop iteration
// ---------------------------------------------------------------------------------
template <bool EPID>
__global__ __launch_bounds__(WG) void k_electron(Params P)
{
    if (gated_off(P, EPID ? QEE : QEP)) return;
    extern __shared__ __align__(16) float lds[];
    __shared__ float s_zl[MAX_LAYERS + 1], s_rho[MAX_LAYERS], s_x0[MAX_PMAT + MAX_LAYERS];
    const int nm = EPID ? P.nl : P.nmat_ph;
    const float *src = P.el_tab + (EPID ? MAX_PMAT : 0) * 3 * NB_EL;
    for (int i = threadIdx.x; i < nm * 3 * NB_EL; i += WG) lds[i] = src[i];
    // after the tables, per wave staging buffers for every kind this kernel appends to
    const unsigned smask = EPID ? (1u << QGE) | (1u << QEE) : (1u << QGP) | (1u << QEP) | (1u << QGE) | (1u << QEE);
    constexpr int nstage = EPID ? 2 : 4;
    Stages S;
    stage_carve(S, (uint32_t *)(lds + nm * 3 * NB_EL) + wave_id() * nstage * stage_words(SBUF_E), smask, SBUF_E);
    if (threadIdx.x <= MAX_LAYERS) s_zl[threadIdx.x] = P.zl[threadIdx.x];
    if (threadIdx.x < MAX_LAYERS) s_rho[threadIdx.x] = P.lrho[threadIdx.x];
    if (threadIdx.x < MAX_PMAT + MAX_LAYERS) s_x0[threadIdx.x] = P.el_x0[threadIdx.x];
    __syncthreads();
    const int kind = EPID ? QEE : QEP;
    const int region = EPID ? 1 : 0;
    const float ln09 = -0.105360515657826301f;   // ln 0.9

    Win win = win_start();
    bool active = false;
    Part p;
    // positions advance in FP64: a 0.1 um nudge must move a particle across a face even
    // 50 cm from the frame origin and at grazing incidence
    double px = 0, py = 0, pz = 0;
    Local L;
    zero(L);
    int nsteps = 0;
    int hpend = 0;   // a hard event pending at p: 1 process not chosen yet, 2 a Moller sample to retry
    int hmat = 0;    // the medium of the step that ended in it
    float hsig = 0.0f;   // the hard cross section its distance was drawn against
    unsigned long long lane_iters = 0, wave_iters = 0;
    for (;;) {
        stage_flush_all(P, S, SBUF_E / 2);
        const bool was = active;
        refill(P, kind, win, active, p);
        const unsigned long long act = __ballot(active);
        if (act == 0) break;
        lane_iters += __popcll(act);
        wave_iters += 64;
        if (active && !was) {
            ++L.items;
            nsteps = 0;
            hpend = 0;
            px = p.x; py = p.y; pz = p.z;
        }
        if (!active) continue;
        if (++nsteps > MAX_E_STEPS || !(p.E == p.E)) {
            atomicOr(P.err, nsteps > MAX_E_STEPS ? ERR_STEPS : ERR_NAN);
            ledger(P, p.hist, (double)p.E);
            active = false;
            continue;
        }
        // One Philox draw per lane and iteration, spent together by the wave: a step uses it for
        // the distance to a hard event, the hinge and the scattering angles; a pending hard event
        // uses it to choose between Moller and bremsstrahlung and for a Moller trial.
        const float4 r = rnd4(p, P);
        float T = p.E;
        bool settle = false;   // the end-of-step checks: cut-off, leaving the region
        bool emit = false;     // a secondary set in motion at p
        uint32_t etype = 0u;
        float eE = 0.0f, eu = 0.0f, ev = 0.0f, ew = 0.0f;
        if (hpend == 0) {
            ++L.steps;
            // current cell and medium
            float rho;
            double lo0, hi0, lo1, hi1, lo2, hi2;
            int m, layer = -1;
            if (!EPID) {
                const int ix = min(max((int)(px * P.iddx), 0), P.nx - 1);
                const int iy = min(max((int)(py * P.iddy), 0), P.ny - 1);
                const int iz = min(max((int)(pz * P.iddz), 0), P.nz - 1);
                const uint32_t word = P.vox[((uint32_t)iz * (uint32_t)P.ny + (uint32_t)iy) * (uint32_t)P.nx + (uint32_t)ix];
                rho = __uint_as_float(word & ~3u);
                m = (int)(word & 3u);
                lo0 = ix * P.ddx; hi0 = lo0 + P.ddx;
                lo1 = iy * P.ddy; hi1 = lo1 + P.ddy;
                lo2 = iz * P.ddz; hi2 = lo2 + P.ddz;
            } else {
                int l = 0;
#pragma unroll
                for (int k = 1; k < MAX_LAYERS; ++k)
                    if (k < P.nl && pz >= (double)s_zl[k]) l = k;
                layer = l;
                m = l;
                rho = s_rho[l];
                lo0 = -P.hx; hi0 = P.hx; lo1 = -P.hy; hi1 = P.hy;
                lo2 = s_zl[l]; hi2 = s_zl[l + 1];
            }
            // distance to the cell faces: the offset to the face is taken in FP64, then the small
            // difference is divided in FP32
            float dg = INFINITY;
            if (p.u != 0.0f) dg = fminf(dg, (float)((p.u > 0.0f ? hi0 : lo0) - px) / p.u);
            if (p.v != 0.0f) dg = fminf(dg, (float)((p.v > 0.0f ? hi1 : lo1) - py) / p.v);
            if (p.w != 0.0f) dg = fminf(dg, (float)((p.w > 0.0f ? hi2 : lo2) - pz) / p.w);
            // a boundary-limited step ends just past the face, so that it never carries this
            // cell's medium into the next one
            const float sg = fmaxf(dg, 0.0f) + NUDGE;
            settle = true;
            if (!(rho > 0.0f)) {
                px += (double)sg * p.u;
                py += (double)sg * p.v;
                pz += (double)sg * p.w;
            } else {
                const float *tab = lds + m * 3 * NB_EL;
                const float lnT = __logf(T);
                const Node n0 = node_of(lnT, P.el_lnT0, P.el_idl, NB_EL);
                const float R0 = lerp_tab(tab, n0);
                const Node n9 = node_of(lnT + ln09, P.el_lnT0, P.el_idl, NB_EL);
                const float R9 = lerp_tab(tab, n9);
                // the distance to a hard event is drawn against the largest hard cross section
                // over the energies this step can reach, [0.9 T0, T0]: the cross section falls
                // and then rises with T, so the larger end value bounds it; the event at the
                // step's end is then real with probability sigma(T1) / sh
                const float sh = fmaxf(lerp_tab(tab + NB_EL, n0), lerp_tab(tab + NB_EL, n9));
                const float s_hard = sh > 0.0f ? -__logf(r.x) / (rho * sh) : INFINITY;
                const float s_de = (R0 - R9) / rho;
                const float s_pix = (EPID && layer == P.scoring) ? P.s_pix : INFINITY;
                const float s = fminf(fminf(s_hard, s_de), fminf(sg, s_pix));
                const bool hard = s_hard <= fminf(s_de, fminf(sg, s_pix));
                float T1;
                if (s == s_de) {
                    T1 = DE_FRAC * T;
                } else {
                    // invert the range table: find j with R[j] <= Rt < R[j+1] between the 0.9 T0 node and T0's
                    const float Rt = R0 - rho * s;
                    int lo = n9.i, hi = n0.i + 1;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (tab[mid] <= Rt) lo = mid; else hi = mid;
                    }
                    const float d = tab[lo + 1] - tab[lo];
                    const float f = d > 0.0f ? fminf(fmaxf((Rt - tab[lo]) / d, 0.0f), 1.0f) : 0.0f;
                    T1 = fminf(__expf(P.el_lnT0 + ((float)lo + f) / P.el_idl), T);
                }
                // hinge point: the step's continuous loss is deposited there, in the layer that
                // holds it
                const double a = (double)(r.y * s);
                px += a * p.u;
                py += a * p.v;
                pz += a * p.w;
                const float dep = T - T1;
                if (P.diag) ledger(P, p.hist, (double)T - (double)T1);
                if (EPID && pz >= (double)s_zl[P.scoring] && pz < (double)s_zl[P.scoring + 1]) {
                    tally(P, p.flags, (float)px, (float)py, dep);
                    ++L.tally;
                }
                if (!(P.mask & 16u)) {
                    const float th = highland(T, rho * s, s_x0[(EPID ? MAX_PMAT : 0) + m]) * sqrtf(-2.0f * __logf(r.z));
                    float sth, cth, sp, cp;
                    __sincosf(th, &sth, &cth);
                    __sincosf(TWO_PI_F * r.w, &sp, &cp);
                    rotate(p.u, p.v, p.w, cth, sth, cp, sp);
                }
                const double bb = (double)s - a;
                px += bb * p.u;
                py += bb * p.v;
                pz += bb * p.w;
                T = T1;
                p.E = T;
                if (hard) {
                    // the event itself takes the next draw, with the rest of the wave
                    hpend = 1;
                    hmat = m;
                    hsig = sh;
                    settle = false;
                }
            }
            p.x = (float)px; p.y = (float)py; p.z = (float)pz;
        } else {
            // the hard event at the end of the previous step (position p, energy T)
            const float *tab = lds + hmat * 3 * NB_EL;
            bool moller = hpend == 2;
            float u1 = r.x, u2 = r.y, uphi = r.z;   // a retried Moller trial
            bool real = true;
            if (hpend == 1) {
                // real with probability sigma(T1) / hsig; the same uniform picks the process
                const Node n1 = node_of(__logf(T), P.el_lnT0, P.el_idl, NB_EL);
                const float sig1 = lerp_tab(tab + NB_EL, n1), fm = lerp_tab(tab + 2 * NB_EL, n1);
                const float sm1 = T > 2.0f * (float)WCUT ? sig1 * fm : 0.0f;   // no Moller event below 2 WCUT
                const float u = r.x * hsig;
                moller = u < sm1;
                real = u < sm1 + (sig1 - sig1 * fm);
                if (moller) ++L.moller; else if (real) ++L.brems;
                u1 = r.y; u2 = r.z; uphi = r.w;
            }
            if (!real) {
                hpend = 0;   // a fictitious event: the electron goes on unchanged
                settle = true;
            } else if (moller) {
                float eps;
                if (moller_trial(moller_setup(T), u1, u2, eps)) {
                    const float W = eps * T, Tp = T - W;
                    const float tt = T + 2.0f * MEC2F;
                    const float cd = fminf(1.0f, sqrtf(W * tt / (T * (W + 2.0f * MEC2F))));
                    const float cq = fminf(1.0f, sqrtf(Tp * tt / (T * (Tp + 2.0f * MEC2F))));
                    float sp, cp;
                    __sincosf(TWO_PI_F * uphi, &sp, &cp);
                    eu = p.u; ev = p.v; ew = p.w;
                    rotate(eu, ev, ew, cd, sqrtf(fmaxf(0.0f, 1.0f - cd * cd)), cp, sp);
                    rotate(p.u, p.v, p.w, cq, sqrtf(fmaxf(0.0f, 1.0f - cq * cq)), -cp, -sp);
                    if (P.diag) ledger(P, p.hist, (double)T - (double)Tp - (double)W);
                    T = Tp;
                    emit = true;
                    etype = 1u;
                    eE = W;
                    hpend = 0;
                    settle = true;
                } else {
                    hpend = 2;
                }
            } else {
                const float k = brems_k(T, u1);
                const float Tn = T - k;
                if (P.diag) ledger(P, p.hist, (double)T - (double)Tn - (double)k);
                T = Tn;
                emit = true;
                etype = 0u;
                eE = k;
                eu = p.u; ev = p.v; ew = p.w;
                hpend = 0;
                settle = true;
            }
            p.E = T;
        }
        if (emit) {
            // the delta ray or bremsstrahlung photon, from one code path
            Part c;
            make_child(p, c, etype);
            c.x = p.x; c.y = p.y; c.z = p.z;
            c.u = eu; c.v = ev; c.w = ew;
            c.E = eE;
            const bool local = etype == 0u ? eE < P.pcut : (!P.coupled || eE < P.ecut);
            if (local) deposit_point(P, region, c, eE, L);
            else place(P, region, c, L, S);
        }
        if (!settle) continue;
        if (T < P.ecut) {
            deposit_point(P, region, p, T, L);
            if ((p.flags & F_TYPE) == 2u) annihilate(P, region, p, L, S);
            active = false;
            continue;
        }
        // where is the end point
        if (!EPID) {
            const bool inside = px >= 0.0 && px < (double)P.Lx && py >= 0.0 && py < (double)P.Ly && pz >= 0.0 &&
                                pz < (double)P.Lz;
            if (!inside) {
                const int rr = vacuum_phantom_frame(P, p);
                if (rr == 0) {
                    px = p.x; py = p.y; pz = p.z;   // re-entered through a face
                } else {
                    if (rr == 1) append(P, S, QEE, true, p);
                    else ledger(P, p.hist, (double)p.E);
                    active = false;
                }
            }
        } else {
            const bool inside = px >= (double)-P.hx && px < (double)P.hx && py >= (double)-P.hy && py < (double)P.hy &&
                                pz >= 0.0 && pz < (double)P.zback;
            if (!inside) {
                ledger(P, p.hist, (double)p.E);
                active = false;
            }
        }
    }
    stage_flush_all(P, S, 1);
    flush_stats(P, L, EPID ? S_ESTEP_E : S_ESTEP_P, kind, lane_iters, wave_iters);
}

template __global__ void k_electron<false>(Params);
template __global__ void k_electron<true>(Params);

// ---------------------------------------------------------------------------------
// tally folding, image, sigma-bar, diagnostics
// ---------------------------------------------------------------------------------
struct FoldArgs {
    double nb[MAX_SLOTS];   // histories of each batch to fold
    int slot[MAX_SLOTS];    // its image slot; batches are listed (and added) in batch order
    int n;
};

__global__ void k_fold(Params P, FoldArgs A)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P.npix; i += gridDim.x * blockDim.x) {
        double s = P.sum[i], s2 = P.sum2[i];
        for (int j = 0; j < A.n; ++j) {
            const size_t k = (size_t)A.slot[j] * P.npix + i;
            double v;
            if (P.tally_mode == 1) {
                const unsigned long long q = ((unsigned long long *)P.img)[k];
                if (q >= (1ull << 62)) atomicOr(P.err, ERR_FIXED);
                v = (double)q * (1.0 / 4294967296.0);
                ((unsigned long long *)P.img)[k] = 0;
            } else {
                v = ((double *)P.img)[k];
                ((double *)P.img)[k] = 0.0;
            }
            s += v;
            s2 += v * v / A.nb[j];
        }
        P.sum[i] = s;
        P.sum2[i] = s2;
    }
}

// Kahan mode: reduce deposit records into the slot images without atomics on the image, in
// an order that does not depend on scheduling, so that the image is the same on every run.
// Records are binned by image element with a counting sort (arbitrary order within an
// element), each element's records are then put in ascending order (a canonical order of the
// same multiset of values), and one workgroup per tile of KT consecutive elements reduces the
// tile's records in LDS to Kahan-compensated FP32 partials and the partials to the image.
__global__ void k_rec_count(const uint32_t *pix, uint32_t n, uint32_t *count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(&count[pix[i]], 1u);
}

// exclusive scan in place, three phases: block sums, scan of block sums, add
__global__ void k_scan_blocks(uint32_t *a, uint32_t n, uint32_t *bsum)
{
    __shared__ uint32_t s[1024];
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = i < n ? a[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) a[i] = s[threadIdx.x] - v;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

__global__ void k_scan_top(uint32_t *bsum, uint32_t nb)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t b = 0; b < nb; ++b) { const uint32_t t = bsum[b]; bsum[b] = acc; acc += t; }
    }
}

__global__ void k_scan_add(uint32_t *a, uint32_t n, const uint32_t *bsum)
{
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n) a[i] += bsum[blockIdx.x];
}

__global__ void k_rec_scatter(const uint32_t *pix, const float *e, uint32_t n, uint32_t *cursor, float *sorted)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t k = atomicAdd(&cursor[pix[i]], 1u);
        sorted[k] = e[i];
    }
}

// each element's records [start, end) into ascending order, in place (heapsort: no extra
// memory, n log n even for a pixel that collects many records).  Deposits are positive, so
// their bit patterns order like their values.
__global__ void k_rec_order(const uint32_t *start, const uint32_t *end, float *sorted, uint32_t nimg)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nimg; i += gridDim.x * blockDim.x) {
        uint32_t *a = (uint32_t *)sorted + start[i];
        const uint32_t n = end[i] - start[i];
        if (n < 2) continue;
        auto sift = [&](uint32_t root, uint32_t lim) {
            const uint32_t v = a[root];
            while (2 * root + 1 < lim) {
                uint32_t ch = 2 * root + 1;
                if (ch + 1 < lim && a[ch + 1] > a[ch]) ++ch;
                if (a[ch] <= v) break;
                a[root] = a[ch];
                root = ch;
            }
            a[root] = v;
        };
        for (uint32_t r = n / 2; r-- > 0;) sift(r, n);
        for (uint32_t m = n - 1; m > 0; --m) {
            const uint32_t t = a[0];
            a[0] = a[m];
            a[m] = t;
            sift(0, m);
        }
    }
}

constexpr int KT = 256;                   // image elements per tile (one workgroup)
constexpr int KSL = 8;                    // records per thread slice
constexpr int KCHUNK = KT * KSL;          // records staged in LDS per round

__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// One workgroup per tile of KT consecutive image elements, whose records are contiguous,
// [start[t0], end[t0 + KT - 1]).  The records pass through LDS in chunks of KCHUNK; in each
// chunk thread j owns the fixed slice of records [j * KSL, (j + 1) * KSL) and forms a
// Kahan-compensated FP32 partial for every run of one element's records inside its slice
// (kept in LDS at the position of the run's last record); then the thread of each element
// adds its element's partials in slice order into its own compensated sum.  An element with
// many records is thus summed by many threads at once, and every step has a fixed order, so
// the tile's partials reduce to the same image on every run.
__global__ __launch_bounds__(KT) void k_rec_kahan(const uint32_t *start, const uint32_t *end, const float *sorted,
                                                  uint32_t nimg, double *img)
{
    __shared__ float chunk[KCHUNK];
    __shared__ float2 part[KCHUNK];
    __shared__ uint32_t st[KT + 1];      // record offsets of the tile's elements, st[KT] = tile end
    const uint32_t t0 = blockIdx.x * KT, i = t0 + threadIdx.x;
    const uint32_t last = min(t0 + KT, nimg) - 1;
    const uint32_t b0 = start[t0], b1 = end[last];
    if (b1 == b0) return;   // uniform over the workgroup
    st[threadIdx.x] = i < nimg ? start[i] : b1;
    if (threadIdx.x == 0) st[KT] = b1;
    const uint32_t my0 = i < nimg ? start[i] : 0, my1 = i < nimg ? end[i] : 0;
    float S = 0.0f, C = 0.0f;
    for (uint32_t base = b0; base < b1; base += KCHUNK) {
        const uint32_t lim = min(base + (uint32_t)KCHUNK, b1);
        __syncthreads();   // st written; the previous chunk's partials consumed
        for (uint32_t k = base + threadIdx.x; k < lim; k += KT) chunk[k - base] = sorted[k];
        __syncthreads();
        // slice partials
        const uint32_t k0 = base + threadIdx.x * KSL, k1 = min(k0 + (uint32_t)KSL, lim);
        if (k0 < k1) {
            uint32_t lo = 0, hi = KT;   // the element of record k0: the last e with st[e] <= k0
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (st[mid] <= k0) lo = mid; else hi = mid;
            }
            uint32_t e = lo;
            float s = 0.0f, c = 0.0f;
            for (uint32_t k = k0; k < k1; ++k) {
                if (k >= st[e + 1]) {
                    part[k - 1 - base] = make_float2(s, c);
                    s = 0.0f;
                    c = 0.0f;
                    while (k >= st[e + 1]) ++e;
                }
                kahan_add(s, c, chunk[k - base]);
            }
            part[k1 - 1 - base] = make_float2(s, c);
        }
        __syncthreads();
        // the element's partials, slice by slice
        const uint32_t lo = max(my0, base), hi = min(my1, lim);
        if (lo < hi) {
            for (uint32_t q = (lo - base) / KSL; q <= (hi - 1 - base) / KSL; ++q) {
                const uint32_t kl = min(hi, base + (q + 1) * (uint32_t)KSL) - 1;
                const float2 p = part[kl - base];
                kahan_add(S, C, p.x - p.y);
            }
        }
    }
    if (i < nimg && my1 > my0) img[i] += (double)S - (double)C;
}

__global__ void k_image(Params P, double n, double nbatch, double *mean, double *var)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P.npix; i += gridDim.x * blockDim.x) {
        const double s = P.sum[i], s2 = P.sum2[i];
        mean[i] = s / n;
        const double v = (nbatch > 1.0) ? (s2 - s * s / n) / (n * (nbatch - 1.0)) : 0.0;
        var[i] = v > 0.0 ? v : 0.0;
    }
}

// one block: max of the mean, then the mean of sigma/D over pixels above threshold
__global__ void k_sigma_bar(Params P, double n, double nbatch, double thr, double *out)
{
    __shared__ double red[1024];
    __shared__ double cnt[1024];
    double mx = 0.0;
    for (uint32_t i = threadIdx.x; i < P.npix; i += blockDim.x) mx = fmax(mx, P.sum[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double cut = thr * red[0];
    __syncthreads();
    double acc = 0.0, c = 0.0;
    for (uint32_t i = threadIdx.x; i < P.npix; i += blockDim.x) {
        const double s = P.sum[i];
        if (s > 0.0 && s >= cut) {
            const double m = s / n;
            double v = (nbatch > 1.0) ? (P.sum2[i] - s * s / n) / (n * (nbatch - 1.0)) : 0.0;
            v = v > 0.0 ? v : 0.0;
            acc += sqrt(v) / m;
            c += 1.0;
        }
    }
    red[threadIdx.x] = acc;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            red[threadIdx.x] += red[threadIdx.x + o];
            cnt[threadIdx.x] += cnt[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = cnt[0] > 0 ? red[0] / cnt[0] : INFINITY;
}

// per-history ledger check: residual = |E_in - sum of ledger| / E_in
__global__ void k_diag_check(Params P, uint32_t nh, unsigned long long *maxbits, double *sums)
{
    double ein = 0.0, led = 0.0, mx = 0.0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += gridDim.x * blockDim.x) {
        const double a = P.ein[i], b = P.led[i];
        ein += a;
        led += b;
        if (a > 0.0) mx = fmax(mx, fabs(a - b) / a);
        P.led[i] = 0.0;
    }
    atomicMax(maxbits, (unsigned long long)__double_as_longlong(mx));
    unsafeAtomicAdd(&sums[0], ein);
    unsafeAtomicAdd(&sums[1], led);
}

// Start of a queue pass: workgroup 0 adds up the input set's segment fills per kind
// (clamped to the segment capacity; wave k sums queue k, one lane per segment) into
// tot[0..NQ-1] and copies the error word to tot[NQ], so that the host reads both back at
// once; every workgroup also clears its share of the other set's fill counters and of the
// consume heads (n16 16-byte words each), which the pass's appends and claims start from.
static_assert(NSEG == 64 && WG == 64 * NQ, "one lane per segment, one wave per queue");
__global__ void k_pass_start(Params P, const uint32_t *cnt, uint32_t *tot, uint4 *fills, uint4 *heads, uint32_t n16,
                             uint32_t *hist)
{
    if (blockIdx.x == 0) {
        const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
        uint32_t v = min(cnt[((uint32_t)k * NSEG + lane) * CSTRIDE], P.segcap[k]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) {
            tot[k] = v;
            if (hist) hist[k] = v;   // kept per pass, for the host to read after device-driven passes
        }
        if (threadIdx.x == 0) {
            tot[NQ] = *P.err;
            if (hist) hist[NQ] = tot[NQ];
        }
    }
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += gridDim.x * blockDim.x) {
        fills[i] = z;
        heads[i] = z;
    }
}

__global__ void k_zero_u32(uint32_t *a, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = 0;
}
__global__ void k_zero_u64(unsigned long long *a, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = 0;
}

// ---------------------------------------------------------------------------------
// dose-response correction (Sec. 2.2, Sec. 3.1)
// ---------------------------------------------------------------------------------
// Radiological thickness of the phantom along each pixel's ray (Sec. 2.2, item 1): the line
// integral of the density over 1 g/cm^3, from the point source to the pixel centre on the
// scoring layer's mid-plane (or along +z through the centre for a parallel beam).  One thread
// per pixel walks the voxels with the incremental Amanatides-Woo traversal in FP64; the 64
// rays of a wave are 64 neighbouring pixels of a row, so they cross nearly the same voxels.
__global__ __launch_bounds__(256) void k_radthick(RadArgs A)
{
    const uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= (uint32_t)A.npx_u * (uint32_t)A.npx_v) return;
    const uint32_t u = pix % (uint32_t)A.npx_u, v = pix / (uint32_t)A.npx_u;
    const double x = -A.hx + (u + 0.5) * A.pu, y = -A.hy + (v + 0.5) * A.pv;
    // the segment S -> T in the phantom's frame (minimum corner at the origin)
    double S[3], d[3];
    if (A.parallel) {
        S[0] = x - A.ox; S[1] = y - A.oy; S[2] = -1.0;
        d[0] = 0.0; d[1] = 0.0; d[2] = A.nz * A.dz + 2.0;
    } else {
        S[0] = A.sx - A.ox; S[1] = A.sy - A.oy; S[2] = A.sz - A.oz;
        d[0] = x - A.sx; d[1] = y - A.sy; d[2] = A.zt - A.sz;
    }
    const int n[3] = {A.nx, A.ny, A.nz};
    const double h[3] = {A.dx, A.dy, A.dz};
    double amin = 0.0, amax = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double hi = n[a] * h[a];
        if (d[a] == 0.0) {
            if (S[a] < 0.0 || S[a] >= hi) amax = -1.0;   // parallel to the slab and outside it
        } else {
            double a1 = -S[a] / d[a], a2 = (hi - S[a]) / d[a];
            if (a1 > a2) { const double t = a1; a1 = a2; a2 = t; }
            amin = fmax(amin, a1);
            amax = fmin(amax, a2);
        }
    }
    double sum = 0.0;
    if (amax > amin) {
        // the voxel at the entry point, and per axis the parameter of the next plane crossing
        int i[3], step[3];
        double tmax[3], tdel[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double e = S[a] + amin * d[a];
            i[a] = min(max((int)floor(e / h[a]), 0), n[a] - 1);
            step[a] = d[a] > 0.0 ? 1 : (d[a] < 0.0 ? -1 : 0);
            if (step[a] != 0) {
                tmax[a] = ((i[a] + (step[a] > 0 ? 1 : 0)) * h[a] - S[a]) / d[a];
                tdel[a] = h[a] / fabs(d[a]);
            } else {
                tmax[a] = INFINITY;
                tdel[a] = INFINITY;
            }
        }
        double al = amin;
        const int limit = A.nx + A.ny + A.nz + 3;   // a straight line crosses at most this many voxels
        for (int it = 0; it < limit; ++it) {
            const int a = tmax[0] <= tmax[1] ? (tmax[0] <= tmax[2] ? 0 : 2) : (tmax[1] <= tmax[2] ? 1 : 2);
            const double next = fmin(tmax[a], amax);
            if (next > al) {
                const uint32_t word = A.vox[((uint32_t)i[2] * (uint32_t)A.ny + (uint32_t)i[1]) * (uint32_t)A.nx + (uint32_t)i[0]];
                sum += (double)__uint_as_float(word & ~3u) * (next - al);
                al = next;
            }
            if (al >= amax) break;
            i[a] += step[a];
            if (i[a] < 0 || i[a] >= n[a]) break;
            tmax[a] += tdel[a];
        }
        sum *= sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    A.out[pix] = sum;   // g/cm^2 over 1 g/cm^3
}

// Dose-response correction (Sec. 3.1, Eq. 2): out = k(t, s) * image.  For one field s is
// fixed, so the bilinear table lookup is a linear one in t on the two table rows that bracket
// s, blended on the host; the nodes and the blended row are staged in LDS for the search.
__global__ __launch_bounds__(256) void k_response(RespArgs A)
{
    __shared__ double tn[RESP_MAX], row[RESP_MAX];
    if (threadIdx.x < (unsigned)A.nt) {
        tn[threadIdx.x] = A.tn[threadIdx.x];
        row[threadIdx.x] = A.row[threadIdx.x];
    }
    __syncthreads();
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const double t = A.t[p];
    double k;
    if (A.nt == 1 || t <= tn[0]) {
        k = row[0];
    } else if (t >= tn[A.nt - 1]) {
        k = row[A.nt - 1];
    } else {
        int lo = 0, hi = A.nt - 1;   // tn[lo] <= t < tn[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tn[mid] <= t) lo = mid; else hi = mid;
        }
        const double f = (t - tn[lo]) / (tn[hi] - tn[lo]);
        k = (1.0 - f) * row[lo] + f * row[hi];
    }
    A.out[p] = k * A.img[p];
}

// ---------------------------------------------------------------------------------
// building-block probes
// ---------------------------------------------------------------------------------
__global__ void k_dbg_philox(Params P, const uint32_t *ctr, uint32_t *out, unsigned long long n)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 r = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], P.key0, P.key1);
    out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
}

__global__ void k_dbg_sample(Params P, int kind, float p0, float p1, float p2, float *out, unsigned long long n)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Part p;
    p.hist = (uint32_t)i; p.plo = 0x5A5Au; p.phi = (uint32_t)kind; p.draw = 0; p.flags = 0;
    float phu;
    if (kind == 0 || kind == 5) {
        float t;
        const float eps = kn_sample(P, p, p0, t, phu);
        out[i] = kind == 0 ? eps : phu;
    } else if (kind == 1) {
        out[i] = moller_sample(P, p, p0, phu);
    } else if (kind == 2) {
        const float4 r = rnd4(p, P);
        out[i] = brems_k(p0, r.y);
    } else if (kind == 3) {
        const float4 r = rnd4(p, P);
        out[i] = highland(p0, p1, p2) * sqrtf(-2.0f * __logf(r.z));
    }
}

__global__ void k_dbg_table(Params P, int kind, int index, const float *E, float *out, unsigned long long n)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (kind == 0) {
        const Node nd = node_of(__logf(E[i]), P.ph_lnE0, P.ph_idl, NB_PH);
        out[i] = lerp_tab(P.ph_tab + index * 3 * NB_PH, nd);
    } else {
        const Node nd = node_of(__logf(E[i]), P.el_lnT0, P.el_idl, NB_EL);
        out[i] = lerp_tab(P.el_tab + index * 3 * NB_EL + (kind == 2 ? NB_EL : 0), nd);
    }
}

// source probe: the source kernel's own sampling function without transport, for histories
// [h0, h0 + n) (P's key already carries the high-word mix of h0)
__global__ void k_dbg_source(Params P, unsigned long long h0, float *out, unsigned long long n)
{
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Part p;
    float gx = 0, gy = 0, gz = 0;
    uint32_t type = 0;
    source_particle(P, h0 + i, p, gx, gy, gz, type);
    float *o = out + 8 * i;
    o[0] = gx; o[1] = gy; o[2] = gz; o[3] = p.u; o[4] = p.v; o[5] = p.w; o[6] = p.E; o[7] = (float)type;
}

// ---------------------------------------------------------------------------------
// launchers (host side of this translation unit)
// ---------------------------------------------------------------------------------
static inline unsigned grid_for(unsigned long long n, unsigned b) { return (unsigned)((n + b - 1) / b); }


hipError_t launch_source(const Params &P, hipStream_t s)
{
    const unsigned long long n = P.h1 - P.h0;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_source, dim3(grid_for(n, WG)), dim3(WG), 0, s, P);
    return hipGetLastError();
}

size_t lds_bytes(int kind, const Params &P)
{
    switch (kind) {
    case QGP: return (size_t)(WG / 64) * 2 * stage_words(SBUF) * 4;
    case QGE: return (size_t)(WG / 64) * stage_words(SBUF) * 4;
    case QEP: return (size_t)P.nmat_ph * 3 * NB_EL * sizeof(float) + (size_t)(WG / 64) * 4 * stage_words(SBUF_E) * 4;
    default: return (size_t)P.nl * 3 * NB_EL * sizeof(float) + (size_t)(WG / 64) * 2 * stage_words(SBUF_E) * 4;
    }
}

hipError_t launch_transport(int kind, const Params &P, unsigned blocks, hipStream_t s)
{
    const size_t lds = lds_bytes(kind, P);
    switch (kind) {
    case QGP: hipLaunchKernelGGL(k_photon_phantom, dim3(blocks), dim3(WG), lds, s, P); break;
    case QGE: hipLaunchKernelGGL(k_photon_epid, dim3(blocks), dim3(WG), lds, s, P); break;
    case QEP: hipLaunchKernelGGL(k_electron<false>, dim3(blocks), dim3(WG), lds, s, P); break;
    default: hipLaunchKernelGGL(k_electron<true>, dim3(blocks), dim3(WG), lds, s, P); break;
    }
    return hipGetLastError();
}

hipError_t set_lds_limits()
{
    // allow the dynamic LDS sizes above the default 64 KiB cap
    hipError_t e = hipSuccess;
    const int big = 160 * 1024;
    e = hipFuncSetAttribute((const void *)k_photon_phantom, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_photon_epid, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_electron<false>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_electron<true>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

hipError_t launch_fold(const Params &P, const int *slots, const double *nb, int n, hipStream_t s)
{
    FoldArgs A;
    for (int i = 0; i < MAX_SLOTS; ++i) {
        A.nb[i] = i < n ? nb[i] : 1.0;
        A.slot[i] = i < n ? slots[i] : 0;
    }
    A.n = n;
    hipLaunchKernelGGL(k_fold, dim3(min(grid_for(P.npix, 256), 4096u)), dim3(256), 0, s, P, A);
    return hipGetLastError();
}

hipError_t launch_kahan_reduce(const Params &P, uint32_t nrec, uint32_t nimg, uint32_t *count, uint32_t *cursor,
                               uint32_t *bsum, float *sorted, hipStream_t s)
{
    if (nrec == 0) return hipSuccess;
    const unsigned g = min(grid_for(nimg, 256), 8192u);
    hipLaunchKernelGGL(k_zero_u32, dim3(g), dim3(256), 0, s, count, (size_t)nimg);
    hipLaunchKernelGGL(k_rec_count, dim3(min(grid_for(nrec, 256), 8192u)), dim3(256), 0, s, P.rec_pix, nrec, count);
    const unsigned nb = grid_for(nimg, 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, count, nimg, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(64), 0, s, bsum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, count, nimg, bsum);
    // count now holds segment starts; cursor (a copy) advances to the segment ends
    const hipError_t e = hipMemcpyAsync(cursor, count, (size_t)nimg * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rec_scatter, dim3(min(grid_for(nrec, 256), 8192u)), dim3(256), 0, s, P.rec_pix, P.rec_e,
                       nrec, cursor, sorted);
    hipLaunchKernelGGL(k_rec_order, dim3(g), dim3(256), 0, s, count, cursor, sorted, nimg);
    hipLaunchKernelGGL(k_rec_kahan, dim3(grid_for(nimg, KT)), dim3(KT), 0, s, count, cursor, sorted, nimg, (double *)P.img);
    return hipGetLastError();
}

hipError_t launch_image(const Params &P, double n, double nb, double *mean, double *var, hipStream_t s)
{
    hipLaunchKernelGGL(k_image, dim3(min(grid_for(P.npix, 256), 4096u)), dim3(256), 0, s, P, n, nb, mean, var);
    return hipGetLastError();
}

hipError_t launch_sigma_bar(const Params &P, double n, double nb, double thr, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sigma_bar, dim3(1), dim3(1024), 0, s, P, n, nb, thr, out);
    return hipGetLastError();
}

hipError_t launch_diag_check(const Params &P, uint32_t nh, unsigned long long *maxbits, double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_check, dim3(min(grid_for(nh, 256), 2048u)), dim3(256), 0, s, P, nh, maxbits, sums);
    return hipGetLastError();
}

hipError_t launch_radthick(const RadArgs &A, hipStream_t s)
{
    const unsigned n = (unsigned)A.npx_u * (unsigned)A.npx_v;
    hipLaunchKernelGGL(k_radthick, dim3((n + 255) / 256), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_response(const RespArgs &A, hipStream_t s)
{
    hipLaunchKernelGGL(k_response, dim3((A.n + 255) / 256), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_pass_start(const Params &P, const uint32_t *cnt, uint32_t *tot, uint32_t *fills, uint32_t *heads,
                             size_t words, hipStream_t s, uint32_t *hist)
{
    if (words % 4 != 0 || cnt == nullptr || tot == nullptr || fills == nullptr || heads == nullptr) return hipErrorInvalidValue;
    const uint32_t n16 = (uint32_t)(words / 4);
    hipLaunchKernelGGL(k_pass_start, dim3(8), dim3(WG), 0, s, P, cnt, tot, (uint4 *)fills, (uint4 *)heads, n16, hist);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if (bytes % 8 == 0 && ((uintptr_t)p % 8) == 0) {
        const size_t n = bytes / 8;
        hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)min((n + 255) / 256, (size_t)8192)), dim3(256), 0, s,
                           (unsigned long long *)p, n);
    } else {
        const size_t n = (bytes + 3) / 4;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)min((n + 255) / 256, (size_t)8192)), dim3(256), 0, s,
                           (uint32_t *)p, n);
    }
    return hipGetLastError();
}

hipError_t launch_dbg_philox(const Params &P, const uint32_t *ctr, uint32_t *out, unsigned long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_dbg_philox, dim3(grid_for(n, 256)), dim3(256), 0, s, P, ctr, out, n);
    return hipGetLastError();
}

hipError_t launch_dbg_source(const Params &P, unsigned long long h0, float *out, unsigned long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_dbg_source, dim3(grid_for(n, 256)), dim3(256), 0, s, P, h0, out, n);
    return hipGetLastError();
}

hipError_t launch_dbg_sample(const Params &P, int kind, float p0, float p1, float p2, float *out,
                             unsigned long long n, hipStream_t s)
{
    if (kind == 4) {
        return hipErrorInvalidValue;   // the source probe has its own launcher
    } else {
        hipLaunchKernelGGL(k_dbg_sample, dim3(grid_for(n, 256)), dim3(256), 0, s, P, kind, p0, p1, p2, out, n);
    }
    return hipGetLastError();
}

hipError_t launch_dbg_table(const Params &P, int kind, int index, const float *E, float *out, unsigned long long n,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_dbg_table, dim3(grid_for(n, 256)), dim3(256), 0, s, P, kind, index, E, out, n);
    return hipGetLastError();
}

}  // namespace epidmc
