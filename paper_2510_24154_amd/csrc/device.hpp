// device.hpp -- gfx950 building blocks of the transport kernels: the counter-based RNG,
// structure-of-arrays particle queues with wave-aggregated claims and appends, LDS table
// lookups, region geometry, deposits and the tally.
#pragma once
#include "engine.hpp"

namespace epidmc {

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  One call yields four 32-bit
// words.  A particle's stream is keyed by the run seed; its counter is (draw, particle
// id lo, particle id hi, history), so a trajectory never depends on the thread or queue
// slot that carries it.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// open-interval uniform from the top 24 bits: (floor(x / 2^8) + 1/2) 2^-24, never 0 or 1
__device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 8) + 0.5f) * 5.9604644775390625e-8f; }

struct Part {
    float x, y, z, u, v, w, E;
    uint32_t hist, plo, phi, draw, flags;
};

__device__ __forceinline__ float4 rnd4(Part &p, const Params &P)
{
    // the key is a wave-uniform value; hiding it from the optimiser at each call keeps the
    // compiler from hoisting the ten-round key schedule (twenty scalar registers) out of the
    // transport loops, where it would push other uniforms into spill slots: the schedule is
    // recomputed with scalar adds, which issue beside the vector work
    uint32_t k0 = P.key0, k1 = P.key1;
    asm volatile("" : "+s"(k0), "+s"(k1));
    const uint4 r = philox10(p.draw++, p.plo, p.phi, p.hist, k0, k1);
    return make_float4(u01(r.x), u01(r.y), u01(r.z), u01(r.w));
}

// A secondary's particle id: a 64-bit mix of its parent's id and draw counter, after which
// the parent's counter advances.  Siblings get distinct ids (the draw counter differs and the
// mix is a bijection of 64-bit words); ids of unrelated particles of one history coincide
// with probability about n^2 / 2^65.  The mix is the SplitMix64 finaliser (Steele, Lea and
// Flood, OOPSLA 2014); an id only has to be distinct, since Philox decorrelates counters.
__device__ __forceinline__ void make_child(Part &parent, Part &c, uint32_t type)
{
    unsigned long long x = (((unsigned long long)parent.phi << 32) | parent.plo) ^
                           ((unsigned long long)(parent.draw++) * 0x9E3779B97F4A7C15ull);
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    c.hist = parent.hist;
    c.plo = (uint32_t)x;
    c.phi = (uint32_t)(x >> 32);
    c.draw = 0;
    c.flags = (parent.flags & ~(F_TYPE | F_UNSCAT | F_LAYER_MASK)) | type;
}

// ---------------------------------------------------------------------------------
// queues
// ---------------------------------------------------------------------------------
__device__ __forceinline__ Part qload(const Queue &q, uint32_t i)
{
    const uint4 a = q.a[i], b = q.b[i], c = q.c[i];
    Part p;
    p.x = __uint_as_float(a.x); p.y = __uint_as_float(a.y); p.z = __uint_as_float(a.z); p.u = __uint_as_float(a.w);
    p.v = __uint_as_float(b.x); p.w = __uint_as_float(b.y); p.E = __uint_as_float(b.z); p.hist = b.w;
    p.plo = c.x; p.phi = c.y; p.draw = c.z; p.flags = c.w;
    return p;
}

__device__ __forceinline__ void qstore(const Queue &q, uint32_t i, const Part &p)
{
    q.a[i] = make_uint4(__float_as_uint(p.x), __float_as_uint(p.y), __float_as_uint(p.z), __float_as_uint(p.u));
    q.b[i] = make_uint4(__float_as_uint(p.v), __float_as_uint(p.w), __float_as_uint(p.E), p.hist);
    q.c[i] = make_uint4(p.plo, p.phi, p.draw, p.flags);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// the wave's index in its workgroup, as a scalar (wave-uniform) value
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// segment counters: [kind][segment], one 128-byte line each
__device__ __forceinline__ uint32_t *seg_ctr(uint32_t *base, int kind, uint32_t s)
{
    return base + ((uint32_t)kind * NSEG + s) * CSTRIDE;
}

// A wave's home segment.  Workgroups are dealt to the XCDs in turn, so with WG / 64 = 4 waves
// per workgroup and NSEG = 64 every segment is used by the waves of a single XCD.
__device__ __forceinline__ uint32_t home_seg() { return ((uint32_t)blockIdx.x * (WG / 64) + (uint32_t)wave_id()) % NSEG; }

// Append to a next-pass queue: the executing lanes with `pred` set take consecutive slots of
// segment `seg`, one atomic per wave.  Valid in divergent code: the ballot only sees the
// executing lanes and the leader is one of them.  Segments are sized at 1/NSEG of a queue
// whose capacity is several times what a chunk produces, so a full segment means the chunk
// is too large for the workspace: the particle is dropped and the overflow latched.
__device__ __forceinline__ void qappend(const Params &P, int kind, bool pred, const Part &p, uint32_t seg)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0) return;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(seg_ctr(P.cnt_out, kind, seg), (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (pred) {
        const uint32_t i = base + (uint32_t)__popcll(m & __lanemask_lt());
        if (i < P.segcap[kind]) qstore(P.out[kind], seg * P.segcap[kind] + i, p);
        else atomicOr(P.err, ERR_QUEUE);
    }
}

// ---------------------------------------------------------------------------------
// LDS staging of appends: device-scope atomics on one queue counter are the scarce
// resource (they serialise beyond the XCD caches), so a kernel whose lanes append often
// stages particles in a per-wave LDS buffer and appends them to the global queue in bulk.
// ---------------------------------------------------------------------------------
// A wave's staging buffers, one per queue kind that the kernel appends to often (null:
// append straight to the queue).  A buffer holds `sb` particles as three arrays of sb
// 16-byte words, then the fill count, then padding to 16 bytes: stage_words(sb) words.
struct Stages {
    uint32_t *w[NQ];
    uint32_t sb;
    uint32_t seg;   // the wave's home segment, where its flushes go
};

__host__ __device__ constexpr int stage_words(int sb) { return 12 * sb + 4; }

__device__ __forceinline__ Stages no_stages() { return Stages{{nullptr, nullptr, nullptr, nullptr}, 0, 0}; }

__device__ __forceinline__ void stage_put(uint32_t *w, uint32_t sb, uint32_t i, const Part &p)
{
    uint4 *w4 = (uint4 *)w;
    w4[i] = make_uint4(__float_as_uint(p.x), __float_as_uint(p.y), __float_as_uint(p.z), __float_as_uint(p.u));
    w4[sb + i] = make_uint4(__float_as_uint(p.v), __float_as_uint(p.w), __float_as_uint(p.E), p.hist);
    w4[2 * sb + i] = make_uint4(p.plo, p.phi, p.draw, p.flags);
}

__device__ __forceinline__ void stage_copy(const Queue &q, uint32_t g, const uint32_t *w, uint32_t sb, uint32_t i)
{
    const uint4 *w4 = (const uint4 *)w;
    q.a[g] = w4[i];
    q.b[g] = w4[sb + i];
    q.c[g] = w4[2 * sb + i];
}

// append one particle per lane with `pred`, through the wave's staging buffer when the kind
// has one; valid in divergent code (the slot comes from an LDS atomic); a full buffer spills
// straight to the queue
__device__ __forceinline__ void append(const Params &P, const Stages &S, int kind, bool pred, const Part &p)
{
    uint32_t *w = S.w[kind];
    if (!w) {
        qappend(P, kind, pred, p, home_seg());
        return;
    }
    if (!pred) return;
    const uint32_t i = __hip_atomic_fetch_add(w + 12 * S.sb, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const bool full = i >= S.sb;
    if (!full) stage_put(w, S.sb, i, p);
    if (__ballot(full)) qappend(P, kind, full, p, home_seg());
}

// move a wave's staged particles of `kind` to the global queue when at least `minfill` are
// waiting; call with the wave converged.
// LDS instructions of one wave complete in order, so the buffer needs no memory fence: the
// fill count is read and reset with wave-scope atomics, and wave barriers keep the compiler
// from moving the staged reads and writes across them (a fence would also wait for every
// outstanding global load and store of the wave).
__device__ __forceinline__ void stage_flush(const Params &P, Stages &S, int kind, uint32_t minfill)
{
    uint32_t *w = S.w[kind];
    if (!w) return;
    __builtin_amdgcn_wave_barrier();
    const uint32_t n =
        min(__hip_atomic_load(w + 12 * S.sb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT), S.sb);
    if (n == 0 || n < minfill) return;
    // one reservation in the wave's home segment (a full segment: see qappend)
    const uint32_t cap = P.segcap[kind];
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(seg_ctr(P.cnt_out, kind, S.seg), n);
    base = __shfl(base, 0);
    const uint32_t fit = base < cap ? min(n, cap - base) : 0u;
    for (uint32_t i = lane_id(); i < fit; i += 64) stage_copy(P.out[kind], S.seg * cap + base + i, w, S.sb, i);
    if (fit < n && lane_id() == 0) atomicOr(P.err, ERR_QUEUE);
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) __hip_atomic_store(w + 12 * S.sb, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __builtin_amdgcn_wave_barrier();
}

// flush every staged kind (at least `minfill` waiting); wave converged
__device__ __forceinline__ void stage_flush_all(const Params &P, Stages &S, uint32_t minfill)
{
#pragma unroll
    for (int k = 0; k < NQ; ++k) stage_flush(P, S, k, minfill);
}

// carve a wave's staging buffers for the kinds in `mask` out of LDS at `base` (16-byte
// aligned) and clear their fill counts; returns the words used
__device__ __forceinline__ int stage_carve(Stages &S, uint32_t *base, unsigned mask, uint32_t sb)
{
    S = no_stages();
    S.sb = sb;
    S.seg = home_seg();
    int used = 0;
#pragma unroll
    for (int k = 0; k < NQ; ++k)
        if (mask & (1u << k)) {
            S.w[k] = base + used;
            if (lane_id() == 0) S.w[k][12 * sb] = 0;
            used += stage_words(sb);
        }
    return used;
}

// Wave-uniform window [b, e) of queue items (absolute indices) claimed WIN at a time from
// segment `seg`; a wave starts at its home segment and moves through the others as they
// run dry, so the waves share the work to the end with claims spread over NSEG counters.
struct Win {
    uint32_t b, e, seg, tried;
    int done;
};

__device__ __forceinline__ Win win_start() { return Win{0u, 0u, home_seg(), 0u, 0}; }

constexpr uint32_t NO_ITEM = 0xFFFFFFFFu;

// next window of queue `kind`, or done
__device__ __forceinline__ void next_window(const Params &P, int kind, Win &win)
{
    const uint32_t cap = P.segcap[kind];
    while (!win.done) {
        const uint32_t ns = min((uint32_t)__builtin_amdgcn_readfirstlane(*seg_ctr(P.cnt_in, kind, win.seg)), cap);
        uint32_t *head = seg_ctr(P.heads, kind, win.seg);
        // a plain read first: an exhausted segment costs no atomic
        uint32_t b = __builtin_amdgcn_readfirstlane(__hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (b < ns) {
            if (lane_id() == 0) b = atomicAdd(head, (uint32_t)WIN);
            b = __shfl(b, 0);
        }
        if (b < ns) {
            win.b = win.seg * cap + b;
            win.e = win.seg * cap + min(b + (uint32_t)WIN, ns);
            return;
        }
        if (++win.tried == NSEG) win.done = 1;
        else win.seg = (win.seg + 1) % NSEG;
    }
}

// Give the lanes of a converged wave that `want` an item consecutive unclaimed items of
// queue `kind`; returns this lane's item or NO_ITEM when the queue is exhausted.
__device__ __forceinline__ uint32_t claim(const Params &P, int kind, Win &win, bool want)
{
    uint32_t item = NO_ITEM;
    unsigned long long need = __ballot(want);
    while (need) {
        if (win.b >= win.e) {
            next_window(P, kind, win);
            if (win.done) break;
        }
        const uint32_t avail = win.e - win.b;
        const uint32_t rank = (uint32_t)__popcll(need & __lanemask_lt());
        if (((need >> lane_id()) & 1ull) && rank < avail) item = win.b + rank;
        win.b += min((uint32_t)__popcll(need), avail);
        need = __ballot(want && item == NO_ITEM);
    }
    return item;
}

// Give every idle lane of a converged wave the next unclaimed particle of queue `kind`.
__device__ __forceinline__ void refill(const Params &P, int kind, Win &win, bool &active, Part &p)
{
    const uint32_t i = claim(P, kind, win, !active);
    if (i != NO_ITEM) {
        p = qload(P.in[kind], i);
        active = true;
    }
}

// ---------------------------------------------------------------------------------
// tables: node i at ln E0 + i / idl; linear interpolation in ln E
// ---------------------------------------------------------------------------------
struct Node {
    int i;
    float f;
};
__device__ __forceinline__ Node node_of(float lnE, float lnE0, float idl, int nb)
{
    float t = (lnE - lnE0) * idl;
    t = fminf(fmaxf(t, 0.0f), (float)(nb - 1) - 1e-3f);
    Node n;
    n.i = (int)t;
    n.f = t - (float)n.i;
    return n;
}
__device__ __forceinline__ float lerp_tab(const float *t, Node n) { return fmaf(n.f, t[n.i + 1] - t[n.i], t[n.i]); }

// ---------------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool in_phantom(const Params &P, float x, float y, float z)
{
    return x >= 0.0f && x < P.Lx && y >= 0.0f && y < P.Ly && z >= 0.0f && z < P.Lz;
}

__device__ __forceinline__ int epid_layer(const Params &P, float x, float y, float z)
{
    if (!(x >= -P.hx && x < P.hx && y >= -P.hy && y < P.hy)) return -1;
    if (!(z >= 0.0f && z < P.zback)) return -1;
    int l = 0;
#pragma unroll
    for (int k = 1; k < MAX_LAYERS; ++k)
        if (k < P.nl && z >= P.zl[k]) l = k;
    return l;
}

// rotate the unit vector (u,v,w) by polar angle (ct, st) and azimuth (cp, sp)
__device__ __forceinline__ void rotate(float &u, float &v, float &w, float ct, float st, float cp, float sp)
{
    const float s2 = fmaf(-w, w, 1.0f);
    float nu, nv, nw;
    if (s2 > 1e-10f) {
        const float is = rsqrtf(s2), s = s2 * is;
        nu = u * ct + st * (u * w * cp - v * sp) * is;
        nv = v * ct + st * (v * w * cp + u * sp) * is;
        nw = w * ct - st * cp * s;
    } else {
        nu = st * cp;
        nv = st * sp;
        nw = (w >= 0.0f ? ct : -ct);
    }
    const float r = rsqrtf(nu * nu + nv * nv + nw * nw);
    u = nu * r; v = nv * r; w = nw * r;
}

// ---------------------------------------------------------------------------------
// deposits
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void ledger(const Params &P, uint32_t hist, double e)
{
    if (P.diag) atomicAdd(&P.led[hist - (uint32_t)P.h0], e);
}

__device__ __forceinline__ void tally(const Params &P, uint32_t flags, float x, float y, float e)
{
    const float fu = floorf((x + P.hx) * P.ipu), fv = floorf((y + P.hy) * P.ipv);
    if (!(fu >= 0.0f && fu < (float)P.npx_u && fv >= 0.0f && fv < (float)P.npx_v) || !(e > 0.0f)) return;
    const uint32_t pix = (uint32_t)fv * (uint32_t)P.npx_u + (uint32_t)fu;
    const uint32_t slot = flags >> F_SLOT_SHIFT;
    if (P.tally_mode == 0) {
        unsafeAtomicAdd((double *)P.img + (size_t)slot * P.npix + pix, (double)e);
    } else if (P.tally_mode == 1) {
        const long long q = __double2ll_rn((double)e * 4294967296.0);
        atomicAdd((unsigned long long *)P.img + (size_t)slot * P.npix + pix, (unsigned long long)q);
    } else {
        const unsigned long long m = __ballot(1);
        const int leader = __ffsll((long long)m) - 1;
        uint32_t base = 0;
        if ((int)lane_id() == leader) base = atomicAdd(&P.cnt[3 * NQ], (uint32_t)__popcll(m));
        base = __shfl(base, leader);
        const uint32_t i = base + (uint32_t)__popcll(m & __lanemask_lt());
        if (i < P.rec_cap) {
            P.rec_pix[i] = slot * P.npix + pix;
            P.rec_e[i] = e;
        } else {
            atomicOr(P.err, ERR_QUEUE);
        }
    }
}

// point deposit in the EPID located by position (tallied in the scoring layer)
__device__ __forceinline__ void deposit_epid_point(const Params &P, const Part &p, float e, unsigned &ntally)
{
    if (epid_layer(P, p.x, p.y, p.z) == P.scoring) {
        tally(P, p.flags, p.x, p.y, e);
        ++ntally;
    }
}

}  // namespace epidmc
