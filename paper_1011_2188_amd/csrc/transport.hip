// Transport kernel: re-traces stored water tracks through a voxel phantom and
// tallies deposited energy (Sections 2.2 and 2.3 of the paper).
//
// Work decomposition: a wave unit is 64 consecutive histories of one spot
// (aligned to multiples of 64), one history per lane; a spot's run starts at
// its device history counter, which a small kernel advances after the launch.  Consecutive histories
// of a spot share a database track in chunks of R (R = 64 by default), so the
// lanes of a wave read the same step record each step: the record loads are
// broadcast loads, and lanes only diverge in the voxel walk - the paper's
// choice of feeding one stored history to a whole thread group (Section 4).
//
// Per history (task 1, Section 2.3): pick the track of the chunk with Philox,
// find the start step where the remaining energy equals the spot energy,
// sample the lateral source position, and enter the phantom box.  Then (task
// 2) each step's water-equivalent length (WEL) is consumed voxel by voxel at
// geometric length WEL / RSP, its energy split over the voxels in proportion
// to the WEL consumed (telescoping rounding to integers), and at the step end
// the direction is deflected by theta * sqrt(sum(w_v * G_v) / WEL) with
// G = RScP / RSP.  Deposits accumulate in a register while the proton stays
// in one voxel and are flushed with a 64-bit integer atomic when it leaves.
//
// Geometry is FP32 with the position kept as (integer voxel, fraction in the
// voxel), so precision does not degrade with the distance from the origin.
// The source sample and the box entry are computed in FP64 once per history.
#include "fdc_device.h"

// Floating-point contraction only within one source expression (explicit fmaf
// stays fused): the walk's rounding is then fixed by the source text, the same
// in every kernel that inlines it, so all launch variants give identical tallies.
#pragma clang fp contract(on)

namespace fdc {

namespace {

constexpr float kInf = __builtin_huge_valf();

// Work of one history (counted with CNT, a debug option): steps started in
// the phantom, non-vacuum voxel pieces, and deposits flushed to a sink.
struct WorkCount {
    uint32_t steps, visits, flushes;
};

struct Lane {
    int i[3];           // voxel
    float f[3];         // position inside the voxel, voxel units, [0, 1]
    float d[3];         // direction (CT frame, unit)
    float b[3];         // direction in the beam frame
    uint32_t v;         // linear voxel index
};

// Per-direction terms of the walk: dv = voxel units per cm along each axis,
// and the coefficients of the distance (cm) to the exit face along an axis as
// a function of the fraction f inside the voxel: t = ta * f + tb, i.e.
// (1 - f) / |dv| moving up, f / |dv| moving down, infinite along an axis not
// travelled.
__host__ __device__ inline void set_direction_terms(const float d[3], const float inv_vox[3], float ta[3],
                                                    float tb[3], float dv[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dv[a] = d[a] * inv_vox[a];
        const float s = fast_rcp(fabsf(dv[a]));
        ta[a] = d[a] > 0.f ? -s : (d[a] < 0.f ? s : 0.f);
        tb[a] = d[a] > 0.f ? s : (d[a] < 0.f ? 0.f : kInf);
    }
}

// A stored step as the walk reads it (16 bytes, converted once when the
// database is loaded): (dx, the step's energy loss in fixed point as the bits
// of an int32, theta * cos(phi), theta * sin(phi)).
__host__ __device__ inline long long step_energy(float4 r)
{
    return (long long)__builtin_bit_cast(int, r.y);
}

// theta and the azimuth's cosine and sine from (theta cos phi, theta sin phi);
// a step without deflection gets azimuth 0
__host__ __device__ inline void polar_terms(float4 r, float &th, float &c, float &s)
{
    const float t2 = r.z * r.z + r.w * r.w;
    const float ir = fast_rsq(t2 > 0.f ? t2 : 1.f);
    th = t2 > 0.f ? t2 * ir : 0.f;
    c = t2 > 0.f ? r.z * ir : 1.f;
    s = t2 > 0.f ? r.w * ir : 0.f;
}

// Turn a unit direction b by polar angle (st = sin, ct = cos) and azimuth
// (cph, sph) about itself, in the frame fixed by b and the beam axis (a
// direction along the axis takes the azimuth from the beam frame's x axis),
// and renormalise.
__host__ __device__ inline void turn_direction(float b[3], float st, float ct, float cph, float sph)
{
    const float u = b[0], vv = b[1], w = b[2];
    const float rho = fast_sqrt(u * u + vv * vv);     // |u|, |v| <= 1: no overflow
    float nu, nv, nw;
    if (rho < 1e-20f) {
        nu = st * cph;
        nv = st * sph;
        nw = (w < 0.f ? -ct : ct);
    } else {
        const float ir = fast_rcp(rho);
        nu = u * ct + st * (u * w * cph - vv * sph) * ir;
        nv = vv * ct + st * (vv * w * cph + u * sph) * ir;
        nw = w * ct - rho * st * cph;
    }
    const float nrm = fast_rsq(nu * nu + nv * nv + nw * nw);
    b[0] = nu * nrm; b[1] = nv * nrm; b[2] = nw * nrm;
}

// Where a voxel visit's deposit goes.  Every sink adds the integer deposit
// `acc` to E[v] and, with the squared-energy tally, q^2 to E2[v] with
// q = (acc + 2^11) >> 12 (the deposit rounded to 2^-12 MeV).
// (Sinks hold the tally pointers by value: read once per unit, they stay in
// registers instead of being re-read from the plan record at every flush.)
template <bool VAR>
struct GlobalSink {            // 64-bit device atomics straight into the plan's tallies
    unsigned long long *E, *E2;
    __device__ void add(uint32_t v, uint32_t, long long acc) const
    {
        add_global(E + v, (unsigned long long)acc);
        if (VAR) {
            const unsigned long long q = (unsigned long long)((acc + 2048) >> 12);
            add_global(E2 + v, q * q);
        }
    }
};

struct NullSink {              // end-point replays: nothing is tallied
    __host__ __device__ void add(uint32_t, uint32_t, long long) const {}
};

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kProbes = 8;

// Per-workgroup sub-tally in LDS: an open-addressed table of `mask + 1` slots
// (voxel key, energy, squared energy).  A visit adds into the slot holding its
// voxel, claiming an empty one with a compare-and-swap; after kProbes occupied
// slots it falls back to the global atomics.  Voxels consecutive in x land in
// consecutive slots, so the end-of-round flush partly coalesces.  The table
// holds voxels of one plan per round; visits of another plan go straight to
// the global atomics.
template <bool VAR>
struct LdsSink {
    unsigned long long *E, *E2; // tallies of the unit's plan
    bool same;                  // the unit's plan is the one whose voxels the table holds
    uint32_t *keys;
    unsigned long long *e, *e2;
    uint32_t mask;
    __device__ void add(uint32_t v, uint32_t ix, long long acc) const
    {
        const unsigned long long q = (unsigned long long)((acc + 2048) >> 12);
        if (!same) {                               // a round straddling two plans
            add_global(E + v, (unsigned long long)acc);
            if (VAR) add_global(E2 + v, q * q);
            return;
        }
        uint32_t row = v - ix;                     // start of the x row
        row ^= row >> 15;
        row *= 0x2c1b3c6du;
        row ^= row >> 12;
        uint32_t s = (row + ix) & mask;
#pragma unroll 1
        for (int p = 0; p < kProbes; ++p) {
            uint32_t k = keys[s];
            if (k == kEmpty) k = atomicCAS(keys + s, kEmpty, v);
            if (k == kEmpty || k == v) {
                atomicAdd(e + s, (unsigned long long)acc);
                if (VAR) atomicAdd(e2 + s, q * q);
                return;
            }
            s = (s + 1) & mask;
        }
        add_global(E + v, (unsigned long long)acc);
        if (VAR) add_global(E2 + v, q * q);
    }
};

// Slot of a voxel in an LDS table of n slots: a hash of the voxel's x row
// plus its x index, so voxels consecutive in x take consecutive slots (the
// flush of a table then partly coalesces).
__device__ inline uint32_t row_slot(uint32_t v, uint32_t ix, uint32_t n)
{
    uint32_t row = v - ix;
    row ^= row >> 15;
    row *= 0x2c1b3c6du;
    row ^= row >> 12;
    uint32_t s = (uint32_t)(((unsigned long long)row * n) >> 32) + ix;
    return s < n ? s : s % n;
}

// Per-workgroup write-back cache of the tallies in LDS.  A slot is one 64-bit
// word per tally: (voxel + 1) in the top 64 - vbits bits, a partial sum in the
// low vbits bits, 0 = empty.  No update retries:
//  - hit (the word read holds the voxel): one atomic add of the deposit;
//  - miss: one atomic exchange installs (voxel, deposit) and the evicted sum
//    goes to the plan's tally with one global atomic, unless it is the same
//    voxel's (another lane installed it first), which is added back in LDS;
//  - if the word changed voxel between the read and the add, the deposit went
//    into another voxel's sum: the lane adds it to its own voxel's tally and
//    subtracts it from the other voxel's (exact in modular integer arithmetic,
//    whenever that sum is flushed);
//  - an add that takes a sum to half its field or beyond exchanges the word
//    with 0 and flushes it.
// Keys only change by exchange, which carries the whole sum with it, so every
// unit of deposit reaches exactly one voxel's tally and the result equals that
// of global atomics alone.  Headroom: a lane whose add took a sum to half the
// field or beyond exchanges the word before its next LDS access, so at most one
// add per lane of the workgroup (<= 1024 = 2^10) lands on a word past that mark
// before it is emptied; every value added in LDS (a deposit or a sum merged
// back) is below 2^(vbits-12), so a sum stays below
// 2^(vbits-1) + 1025 * 2^(vbits-12) < 2^vbits and never carries into the key.
// Larger deposits go straight to the global tally.  A word whose key is 0
// (an add that landed on a just-emptied word) holds no tally: its sum was also
// sent to the lane's own voxel, and flushes skip it.  The cache holds voxels of
// one plan per round; other plans' visits go straight to the global atomics.
template <bool VAR>
struct CacheSink {
    unsigned long long *E, *E2; // tallies of the unit's plan
    bool same;                  // the unit's plan is the one whose voxels the cache holds
    unsigned long long *ce, *ce2;
    uint32_t n;                 // slots
    uint32_t vbits;             // value bits of a word
    uint32_t nvox;              // voxels of the cached plan (valid keys are 1..nvox)

    __device__ void flush_word(unsigned long long *T, unsigned long long w) const
    {
        const uint32_t kv = (uint32_t)(w >> vbits);
        const unsigned long long val = w & ((1ull << vbits) - 1);
        if (kv != 0u && kv <= nvox && val != 0ull) add_global(T + (kv - 1u), val);
    }

    // after the word's atomic returned o: repair a misdirected add, flush a
    // full word, or flush the evicted sum
    __device__ void settle(unsigned long long *c, unsigned long long *T, uint32_t v, unsigned long long key,
                           unsigned long long val, bool hit, unsigned long long o) const
    {
        const unsigned long long vmask = (1ull << vbits) - 1;
        if (!hit) {
            flush_word(T, o);
            return;
        }
        if ((o & ~vmask) != key) {
            add_global(T + v, val);
            const uint32_t kv = (uint32_t)(o >> vbits);
            if (kv != 0u && kv <= nvox) add_global(T + (kv - 1u), 0ull - val);
        }
        if ((o & vmask) + val >= (1ull << (vbits - 1))) flush_word(T, atomicExch(c, 0ull));
    }

    __device__ void add(uint32_t v, uint32_t ix, long long acc) const
    {
        const unsigned long long q = (unsigned long long)((acc + 2048) >> 12);
        if (!same) {                               // a round straddling two plans
            add_global(E + v, (unsigned long long)acc);
            if (VAR) add_global(E2 + v, q * q);
            return;
        }
        const uint32_t s = row_slot(v, ix, n);
        const unsigned long long vmask = (1ull << vbits) - 1;
        const unsigned long long lim = 1ull << (vbits - 12);
        const unsigned long long key = (unsigned long long)(v + 1) << vbits;
        const unsigned long long v1 = (unsigned long long)acc, v2 = q * q;
        // deposits are >= 0 (the database has dE >= 0)
        bool do1 = acc > 0, do2 = VAR && q != 0;
        if (do1 && v1 >= lim) { add_global(E + v, v1); do1 = false; }
        if (do2 && v2 >= lim) { add_global(E2 + v, v2); do2 = false; }
        // the two words side by side: both reads, both atomics, then both settles
        const unsigned long long w1 = do1 ? ce[s] : 0ull, w2 = do2 ? ce2[s] : 0ull;
        const bool hit1 = (w1 & ~vmask) == key, hit2 = (w2 & ~vmask) == key;
        unsigned long long o1 = 0ull, o2 = 0ull;
        if (do1) o1 = hit1 ? atomicAdd(ce + s, v1) : atomicExch(ce + s, key | v1);
        if (do2) o2 = hit2 ? atomicAdd(ce2 + s, v2) : atomicExch(ce2 + s, key | v2);
        // a miss that evicted the same voxel (installed an instant earlier by
        // another lane, typically of the same wave) adds that sum back
        unsigned long long a1 = v1, a2 = v2;
        bool h1 = hit1, h2 = hit2;
        if (do1 && !hit1 && (o1 & ~vmask) == key && (o1 & vmask) < lim) {
            a1 = o1 & vmask;
            h1 = true;
            o1 = atomicAdd(ce + s, a1);
        }
        if (do2 && !hit2 && (o2 & ~vmask) == key && (o2 & vmask) < lim) {
            a2 = o2 & vmask;
            h2 = true;
            o2 = atomicAdd(ce2 + s, a2);
        }
        if (do1) settle(ce + s, E, v, key, a1, h1, o1);
        if (do2) settle(ce2 + s, E2, v, key, a2, h2, o2);
    }
};

// A beam-line device on a spot's way to the phantom (fdc_beam_device), in
// FP64 like the source: the ray from p along d meets the device's upstream
// face at one pixel; a closed pixel, a pixel off the grid, or a face not ahead
// of p stops the history there (returns true).  Through an open pixel with
// compensator thickness T > 0 the track is replayed from step k in a slab of
// the compensator's material until the displacement along the face normal
// reaches T: each piece consumes water-equivalent length at geometric length
// WEL / RSP, the step's energy split uniformly in WEL with the telescoping
// rounding, the deflection at a step end scaled by sqrt(sum w G / WEL) as in a
// voxel.  On return (false) p, d and b (the beam-frame direction) are at the
// exit face, k is the step being replayed there with tau (WEL consumed), dep
// (its energy deposited so far) and g2 (sum w G) of it done, and up holds the
// energy deposited in the compensator (lost to the phantom).  A track that
// ends inside the compensator stops there (true).
__host__ __device__ inline bool beam_device_pass(const TransportArgs &a, const DevDevice &dv, const DevSpot &sp,
                                                 unsigned long long k0, unsigned long long kend, long long cum,
                                                 long long skip, double phi0, double p[3], double d[3], double b[3],
                                                 unsigned long long &k_out, double &tau_out, int &dep_out,
                                                 double &g2_out, long long &up)
{
    double dn = d[0] * dv.nrm[0] + d[1] * dv.nrm[1] + d[2] * dv.nrm[2];
    double t = (dv.o[0] - p[0]) * dv.nrm[0] + (dv.o[1] - p[1]) * dv.nrm[1] + (dv.o[2] - p[2]) * dv.nrm[2];
    if (!(dn > 0.0) || t < 0.0) return true;
    t /= dn;
#pragma unroll
    for (int q = 0; q < 3; ++q) p[q] += t * d[q];
    double ra = 0.0, rb = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        ra += (p[q] - dv.o[q]) * dv.u1[q];
        rb += (p[q] - dv.o[q]) * dv.u2[q];
    }
    const double fi = floor(ra / dv.pitch[0] + 0.5 * (double)dv.npix[0]);
    const double fj = floor(rb / dv.pitch[1] + 0.5 * (double)dv.npix[1]);
    if (fi < 0.0 || fj < 0.0 || fi >= (double)dv.npix[0] || fj >= (double)dv.npix[1]) return true;
    const double thick = dv.pix[(long)fj * dv.npix[0] + (long)fi];
    if (thick < 0.0) return true;
    k_out = k0;
    if (thick == 0.0) return false;
    double z = 0.0;                                     // displacement along the normal in the slab
    for (unsigned long long k = k0; k < kend; ++k) {
        // the step as replayed (the first one cut to the energy left below the spot energy)
        const float4 r = a.steps[k];
        long long e = step_energy(r);
        double w_tot = r.x;
        const double t2 = (double)r.z * r.z + (double)r.w * r.w;
        double th = t2 > 0.0 ? sqrt(t2) : 0.0;
        double cp = t2 > 0.0 ? r.z / th : 1.0, spp = t2 > 0.0 ? r.w / th : 0.0;
        if (k == k0) {
            const long long e_first = cum + e - skip;
            const double f = (double)e_first / (double)e;
            e = e_first;
            w_tot *= f;
            th *= sqrt(f);
            double s0, c0;
            sincos(phi0, &s0, &c0);
            const double c = cp * c0 - spp * s0;
            spp = spp * c0 + cp * s0;
            cp = c;
        }
        double tau = 0.0, g2 = 0.0;
        long long dep = 0;
        bool on_face = false;                           // the step ended exactly on the exit face
        while (tau < w_tot) {
            dn = d[0] * dv.nrm[0] + d[1] * dv.nrm[1] + d[2] * dv.nrm[2];
            double lgeo = dn > 0.0 ? (thick - z) / dn : __builtin_huge_val();
            if (lgeo < 0.0) lgeo = 0.0;
            const double rem = w_tot - tau, wb = lgeo * dv.rsp;
            double w_v, tau_n, move;
            bool exits;
            if (rem <= wb) {
                w_v = rem;
                tau_n = w_tot;
                move = rem / dv.rsp;
                exits = rem == wb;
            } else {
                w_v = wb;
                tau_n = tau + wb;
                move = lgeo;
                exits = true;
            }
            long long cumk = (long long)rint((double)e * (tau_n / w_tot));
            if (tau_n >= w_tot) cumk = e;
            up += cumk - dep;
            dep = cumk;
            g2 += w_v * dv.g;
            tau = tau_n;
#pragma unroll
            for (int q = 0; q < 3; ++q) p[q] += move * d[q];
            z += move * dn;
            if (exits && tau < w_tot) {                 // out through the exit face inside the step
                k_out = k;
                tau_out = tau;
                dep_out = (int)dep;
                g2_out = g2;
                return false;
            }
            on_face = exits;
        }
        // deflection at the end of the step (textbook polar/azimuth rotation)
        const double th2 = th * sqrt(g2 / w_tot);
        const double st = sin(th2), ct = cos(th2);
        const double u = b[0], v = b[1], w = b[2];
        const double rho = sqrt(u * u + v * v);
        double nu, nv, nw;
        if (rho < 1e-20) {
            nu = st * cp;
            nv = st * spp;
            nw = w < 0.0 ? -ct : ct;
        } else {
            nu = u * ct + st * (u * w * cp - v * spp) / rho;
            nv = v * ct + st * (v * w * cp + u * spp) / rho;
            nw = w * ct - rho * st * cp;
        }
        const double l = sqrt(nu * nu + nv * nv + nw * nw);
        b[0] = nu / l; b[1] = nv / l; b[2] = nw / l;
#pragma unroll
        for (int q = 0; q < 3; ++q) d[q] = sp.e1[q] * b[0] + sp.e2[q] * b[1] + sp.d[q] * b[2];
        if (on_face) {                                  // a step ending on the exit face: the next starts beyond it
            k_out = k + 1;
            tau_out = 0.0;
            dep_out = 0;
            g2_out = 0.0;
            return k + 1 >= kend;
        }
    }
    return true;                                        // the track ended in the compensator
}

// wc: the wave's constants, the spot's field matrix (9 floats, row-major) and
// the plan's 1 / voxel size (3), as values known to be the same in every lane
// of the wave (they live in scalar registers, read at step ends without a
// memory access).
// LISTED: the source is a list of protons (Section 2.3, a phase space read from
// a file): history h is the source's proton h mod count, which brings its own
// start point, direction (and with it the frame of the deflections, kept per
// lane) and energy.
// SEC: the database has secondary trajectories (Section 2.2: a stored
// history is the set of its particles' trajectories): a secondary starts at
// the end of one of its track's primary steps, from the point the primary
// reached and its direction there turned by the secondary's emission angles,
// and is replayed after the primary (an end-point replay follows the primary
// only).  Its energy follows that step's in the track's order, so a skip that
// ends inside it drops it and starts at the next primary step whole.
template <bool EP, bool LISTED, bool SEC, bool CNT, class Sink>
__host__ __device__ void replay_history(const TransportArgs &a, const DevSpot &sp, const DevPlan &pl,
                               const float2 *__restrict__ lut, const float *wc, unsigned long long h,
                               uint32_t slot, long long &inc, long long &esc, const Sink &sink, WorkCount &wk)
{
    // ---- task 1: track, start step, source ---------------------------------
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0;
    if (LISTED) {
        const unsigned long long pi = sp.ps_first + h % sp.ps_count;
        q0 = pl.ps[2 * pi];
        q1 = pl.ps[2 * pi + 1];
    }
    const uint32_t first = a.bin_first[sp.bin];
    const uint32_t nb = a.bin_first[sp.bin + 1] - first;
    const unsigned long long c = h / a.R;
    const uint4 xt = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)(c >> 32), sp.spot,
                                              (sp.plan << 4) | kTagTrack), a.seed_lo, a.seed_hi);
    const uint32_t t = first + (uint32_t)(((uint64_t)xt.x * nb) >> 32);
    unsigned long long k = a.track_off[t];
    unsigned long long kend = a.track_off[t + 1];
    long long skip = LISTED ? sp.bin_fp - to_fp(q0.w) : sp.skip;
    long long cum = 0;
    long long e = 0;
    uint32_t j = SEC ? a.sec_first[t] : 0u;          // the track's next secondary
    for (; k < kend; ++k) {
        e = step_energy(a.steps[k]);
        if (cum + e > skip) break;
        cum += e;
        if (SEC) {
            // (a later track's secondaries, and the end marker, never match k)
            while (a.secs[j].kb == k) cum += a.secs[j++].T;
            if (cum > skip) {
                skip = cum;
                ++k;
                break;
            }
        }
    }
    long long I_h = a.track_T[t] - skip;
    if (I_h < 0) I_h = 0;
    inc = I_h;

    const uint4 xs = philox4x32_10(make_uint4((uint32_t)h, (uint32_t)(h >> 32), sp.spot,
                                              (sp.plan << 4) | kTagSource), a.seed_lo, a.seed_hi);
    // lateral offset: Gaussian of standard deviation sigma (Box-Muller), or for
    // sigma < 0 uniform over a disk of radius -sigma (radius^2 uniform): the
    // circular field of Section 2.5
    const double r = sp.sigma >= 0.f ? sqrt(-2.0 * log(u01(xs.x))) : sqrt(u01(xs.x));
    double sa, ca;
    sincos(2.0 * M_PI * u01(xs.y), &sa, &ca);
    const double n1 = r * ca, n2 = r * sa;
    const float phi0 = (a.flags & kFlagRotate) ? (float)(2.0 * M_PI * u01(xs.z)) : 0.f;
    double p[3], dsrc[3];
    float lm[9];                                    // a listed proton's frame, columns e1 e2 d
    if (LISTED) {
        // its own start and direction, no lateral spread; the frame as for a
        // spot: e2 = normalize(d x a), e1 = e2 x d, a = +x if |d_z| >= 0.9 else +z
        const double dl = sqrt((double)q1.x * q1.x + (double)q1.y * q1.y + (double)q1.z * q1.z);
        const double d[3] = {q1.x / dl, q1.y / dl, q1.z / dl};
        const double ax[3] = {fabs(d[2]) >= 0.9 ? 1.0 : 0.0, 0.0, fabs(d[2]) >= 0.9 ? 0.0 : 1.0};
        double e2[3] = {d[1] * ax[2] - d[2] * ax[1], d[2] * ax[0] - d[0] * ax[2], d[0] * ax[1] - d[1] * ax[0]};
        const double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        e2[0] /= l2; e2[1] /= l2; e2[2] /= l2;
        const double e1[3] = {e2[1] * d[2] - e2[2] * d[1], e2[2] * d[0] - e2[0] * d[2], e2[0] * d[1] - e2[1] * d[0]};
        const double q0p[3] = {q0.x, q0.y, q0.z};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            p[q] = q0p[q];
            dsrc[q] = d[q];
            lm[3 * q + 0] = (float)e1[q];
            lm[3 * q + 1] = (float)e2[q];
            lm[3 * q + 2] = (float)d[q];
        }
    } else {
        const double scale = fabs((double)sp.sigma);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            p[q] = sp.pos[q] + scale * (n1 * sp.e1[q] + n2 * sp.e2[q]);
            dsrc[q] = sp.d[q];
        }
    }

    // a beam-line device on the way (aperture, range compensator): the walk
    // then begins where the history leaves it, possibly inside a step
    const unsigned long long k_first = k;
    double bb[3] = {0.0, 0.0, 1.0};                 // beam-frame direction
    double tau0 = 0.0, g20 = 0.0;
    int dep0 = 0;                                   // (the pass's own split of the step; the walk restates it)
    long long up = 0;                               // energy deposited upstream of the phantom
    if (!LISTED && sp.dev >= 0 && a.devices && I_h > 0 && k < kend) {
        unsigned long long kw = k;
        if (beam_device_pass(a, a.devices[sp.dev], sp, k, kend, cum, skip, (double)phi0, p, dsrc, bb, kw, tau0, dep0,
                             g20, up)) {
            esc = I_h;
            if (EP) {
                a.ep_xyz[3 * slot + 0] = (float)p[0];
                a.ep_xyz[3 * slot + 1] = (float)p[1];
                a.ep_xyz[3 * slot + 2] = (float)p[2];
                a.ep_reason[slot] = 3;
            }
            return;
        }
        k = kw;
        // secondaries emitted at step ends inside the device stay there
        if (SEC)
            while (a.secs[j].kb < k) ++j;
    }

    // ray-box entry (FP64); outside the box is vacuum
    double tin = -__builtin_huge_val(), tout = __builtin_huge_val();
    int ax_in = 0;
    bool miss = false;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double lo = pl.org_d[q], hi = pl.org_d[q] + pl.n[q] * pl.vox_d[q];
        if (dsrc[q] == 0.0) {
            miss |= (p[q] < lo || p[q] >= hi);
        } else {
            double t1 = (lo - p[q]) / dsrc[q], t2 = (hi - p[q]) / dsrc[q];
            if (t1 > t2) { const double tt = t1; t1 = t2; t2 = tt; }
            if (t1 > tin) { tin = t1; ax_in = q; }
            tout = fmin(tout, t2);
        }
    }
    miss = miss || !(tin < tout) || tout <= 0.0;
    if (miss || I_h == 0 || k == kend) {
        esc = I_h;
        if (EP) {
            a.ep_xyz[3 * slot + 0] = (float)p[0];
            a.ep_xyz[3 * slot + 1] = (float)p[1];
            a.ep_xyz[3 * slot + 2] = (float)p[2];
            a.ep_reason[slot] = (I_h == 0 || k == kend) ? 0 : 2;
        }
        return;
    }
    if (tin > 0.0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) p[q] += tin * dsrc[q];
    }
    Lane L;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double u = (p[q] - pl.org_d[q]) / pl.vox_d[q];
        if (tin > 0.0 && q == ax_in) u = dsrc[q] > 0.0 ? 0.0 : (double)pl.n[q];  // on the entry face
        double fl = floor(u);
        int i = (int)fl;
        if (u == fl && dsrc[q] < 0.0) i -= 1;     // a boundary point belongs to the voxel entered
        i = min(max(i, 0), pl.n[q] - 1);
        L.i[q] = i;
        L.f[q] = (float)fmin(fmax(u - (double)i, 0.0), 1.0);
        L.d[q] = (float)dsrc[q];
    }
    L.b[0] = (float)bb[0]; L.b[1] = (float)bb[1]; L.b[2] = (float)bb[2];
    // what the walk reads of the plan and spot, as values (not re-read from
    // memory inside the loops, where the tally atomics could alias them)
    const int nx = pl.n[0], ny = pl.n[1], nz = pl.n[2];
    L.v = ((uint32_t)L.i[2] * (uint32_t)ny + (uint32_t)L.i[1]) * (uint32_t)nx + (uint32_t)L.i[0];
    const uint32_t stride[3] = {1u, (uint32_t)nx, (uint32_t)nx * (uint32_t)ny};

    float ta[3], tb[3], dv[3];
    {
        const float iv[3] = {wc[9], wc[10], wc[11]};
        set_direction_terms(L.d, iv, ta, tb, dv);
    }

    // ---- task 2: re-trace the steps -----------------------------------------
    // Loads are issued one use ahead: the material of the voxel across the
    // exit face (it depends on geometry only) before the current voxel's
    // deposit is flushed, and the next step record one step ahead, so no wait
    // for a load also waits for the tally atomics issued before it.
    const uint16_t *__restrict__ vidx = pl.idx;
    long long acc = 0, hdep = 0;
    // secondaries met by the primary (SEC): kb is the step at whose end the
    // next one starts
    struct Branch {
        int i[3];
        float f[3], b[3];
        uint32_t j;
    };
    Branch br[SEC ? kMaxSecPerTrack : 1];
    int nbr = 0, traj = 0;
    unsigned long long kb = SEC ? a.secs[j].kb : 0ull;
    for (;;) {                                      // the primary, then its secondaries
        uint16_t wcur = load_global(vidx, L.v);          // the current voxel's word
        float2 m = lut[hu_index(wcur)];
        bool escaped = false;
        // the partial first step (its remaining energy e_first of the stored e):
        // length f * dx, angle sqrt(f) * theta, azimuth rotated by phi0; a later
        // step (the walk begins behind a compensator) is replayed whole
        float4 rec = a.steps[k];
        e = step_energy(rec);
        int e32 = (int)e;                               // a step's energy fits 32 bits (checked at load)
        float w_tot = rec.x;
        float th, cph, sph;                             // polar angle, cos and sin of the azimuth
        polar_terms(rec, th, cph, sph);
        float inv_w;
        if (k == k_first) {
            const long long e_first = cum + e - skip;
            const float f = ll_to_f(e_first) / ll_to_f(e);
            e32 = (int)e_first;
            w_tot = f * rec.x;
            th *= sqrtf(f);
            inv_w = 1.f / w_tot;
            if (phi0 != 0.f) {                          // the track rotated rigidly about the beam axis
                float s0, c0;
                sincosf(phi0, &s0, &c0);
                const float c = cph * c0 - sph * s0;
                sph = sph * c0 + cph * s0;
                cph = c;
            }
        } else {
            inv_w = fast_rcp(rec.x);
        }
        // a step begun in a compensator continues with what was done of it there;
        // its energy deposited so far is restated in the walk's own arithmetic
        // (the FP32 split the walk applies to the WEL consumed), so that the
        // walk's pieces, which continue that split, are never negative
        float tau = (float)tau0, g2 = (float)g20;
        int dep = tau0 > 0.0 ? min(e32, (int)rintf((float)e32 * (tau * inv_w))) : 0;
        float4 next_rec = rec;
        if (k + 1 < kend) next_rec = a.steps[k + 1];
        if (CNT) ++wk.steps;
        for (;;) {
            const float ef = (float)e32;
            while (tau < w_tot) {
                const uint32_t kskip = vacuum_skip(wcur);
                if (kskip >= 2u) {
                    // Free flight through vacuum: every voxel within kskip - 1 of this
                    // one (per axis, and inside the box) is vacuum, so the proton
                    // crosses that cube in one move - no WEL, no deposit, no
                    // scattering, as voxel by voxel - to the face it reaches first
                    // (ties x -> y -> z); past the box it escapes.
                    const int n3[3] = {nx, ny, nz};
                    int ext[3];
                    float tj = kInf;
                    int axj = 0;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int room = L.d[q] > 0.f ? n3[q] - 1 - L.i[q] : L.i[q];
                        ext[q] = min((int)kskip - 1, room);
                        const float t = fmaf(ta[q], L.f[q], tb[q]) + (float)ext[q] * fabsf(ta[q]);
                        if (t < tj) { tj = t; axj = q; }
                    }
                    bool out = false;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (q == axj) {
                            const int up = L.d[q] > 0.f ? 1 : -1;
                            const int ni = L.i[q] + up * (ext[q] + 1);
                            out = (unsigned)ni >= (unsigned)n3[q];
                            L.i[q] = out ? L.i[q] + up * ext[q] : ni;             // out: stays on the last voxel's
                            L.f[q] = (up > 0) == out ? 1.f : 0.f;                  // exit face, else the entry face
                        } else if (L.d[q] != 0.f) {
                            const float u = fmaf(tj, dv[q], L.f[q]);
                            float fl = floorf(u);
                            fl = L.d[q] > 0.f ? fminf(fmaxf(fl, 0.f), (float)ext[q]) : fmaxf(fminf(fl, 0.f), -(float)ext[q]);
                            L.i[q] += (int)fl;
                            L.f[q] = fminf(fmaxf(u - fl, 0.f), 1.f);
                        }
                    }
                    if (out) {
                        escaped = true;
                        break;
                    }
                    L.v = ((uint32_t)L.i[2] * (uint32_t)ny + (uint32_t)L.i[1]) * (uint32_t)nx + (uint32_t)L.i[0];
                    wcur = load_global(vidx, L.v);
                    m = lut[hu_index(wcur)];
                    continue;
                }
                // distance (cm) to the exit face along each axis; ties go x -> y -> z
                const float tx = fmaf(ta[0], L.f[0], tb[0]);
                const float ty = fmaf(ta[1], L.f[1], tb[1]);
                const float tz = fmaf(ta[2], L.f[2], tb[2]);
                float tmin = tx;
                int ax = 0;
                if (ty < tmin) { tmin = ty; ax = 1; }
                if (tz < tmin) { tmin = tz; ax = 2; }
                // the voxel across that face, and its material index (prefetch)
                const float d_ax = ax == 0 ? L.d[0] : (ax == 1 ? L.d[1] : L.d[2]);
                const int i_ax = ax == 0 ? L.i[0] : (ax == 1 ? L.i[1] : L.i[2]);
                const int n_ax = ax == 0 ? nx : (ax == 1 ? ny : nz);
                const uint32_t st_ax = ax == 0 ? stride[0] : (ax == 1 ? stride[1] : stride[2]);
                const int ni = i_ax + (d_ax > 0.f ? 1 : -1);
                const bool out = (unsigned)ni >= (unsigned)n_ax;
                const uint32_t vn = d_ax > 0.f ? L.v + st_ax : L.v - st_ax;
                const uint16_t idx_n = load_global(vidx, out ? L.v : vn);
                // consume WEL in this voxel: up to the face (wb) or the step's end
                // (rem), whichever comes first.  Written without branches; a vacuum
                // voxel (RSP 0) gives wb = 0: no WEL, no deposit, a full crossing.
                const float rem = w_tot - tau;
                const float wb = tmin * m.x;
                const bool ends = rem <= wb;                 // the step ends in this voxel
                const float w_v = ends ? rem : wb;
                const float tau_n = ends ? w_tot : tau + wb;
                const float move = ends ? rem * fast_rcp(m.x) : tmin;
                const bool cross = ends ? (rem == wb) : true;
                if (CNT) wk.visits += m.x > 0.f ? 1u : 0u;
                const int cumk = tau_n < w_tot ? min(e32, (int)rintf(ef * (tau_n * inv_w))) : e32;
                const int piece = cumk - dep;
                dep = cumk;
                acc += piece;
                hdep += piece;
                g2 += w_v * m.y;
                tau = tau_n;
#pragma unroll
                for (int q = 0; q < 3; ++q) L.f[q] = fminf(fmaxf(L.f[q] + move * dv[q], 0.f), 1.f);
                if (cross) {
                    if (acc != 0) {
                        sink.add(L.v, (uint32_t)L.i[0], acc);
                        if (CNT) ++wk.flushes;
                        acc = 0;
                    }
                    const float f_new = (d_ax > 0.f) == out ? 1.f : 0.f;   // exit face when out, else entry face
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (q == ax) {
                            L.f[q] = f_new;
                            if (!out) L.i[q] = ni;
                        }
                    }
                    if (out) {
                        escaped = true;
                        break;
                    }
                    L.v = vn;
                    wcur = idx_n;
                    m = lut[hu_index(idx_n)];
                }
            }
            if (escaped) break;
            // deflection at the end of the step, scaled by the traversed material
            const float th2 = th * fast_sqrt(g2 * inv_w);
            float st, ct;
            small_sincos(th2, &st, &ct);
            turn_direction(L.b, st, ct, cph, sph);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                L.d[q] = LISTED ? lm[3 * q + 0] * L.b[0] + lm[3 * q + 1] * L.b[1] + lm[3 * q + 2] * L.b[2]
                                : wc[3 * q + 0] * L.b[0] + wc[3 * q + 1] * L.b[1] + wc[3 * q + 2] * L.b[2];
            {
                const float iv[3] = {wc[9], wc[10], wc[11]};
                set_direction_terms(L.d, iv, ta, tb, dv);
            }
            // secondaries that start here: the point and the direction after the
            // deflection, kept until the primary is done
            if (SEC && k == kb) {
                do {
                    Branch &B = br[nbr++];              // at most kMaxSecPerTrack per track (checked at load)
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        B.i[q] = L.i[q];
                        B.f[q] = L.f[q];
                        B.b[q] = L.b[q];
                    }
                    B.j = j;
                    kb = a.secs[++j].kb;
                } while (kb == k);
            }
            // next stored step (its record and terms were loaded one step ahead)
            if (++k >= kend) break;
            if (CNT) ++wk.steps;
            rec = next_rec;
            if (k + 1 < kend) next_rec = a.steps[k + 1];
            w_tot = rec.x;
            polar_terms(rec, th, cph, sph);
            inv_w = fast_rcp(rec.x);
            e32 = (int)step_energy(rec);
            tau = 0.f;
            g2 = 0.f;
            dep = 0;
        }
        if (!escaped && acc != 0) {
            sink.add(L.v, (uint32_t)L.i[0], acc);
            if (CNT) ++wk.flushes;
        }
        acc = 0;
        if (EP) {                                       // the primary's end
#pragma unroll
            for (int q = 0; q < 3; ++q)
                a.ep_xyz[3 * slot + q] = (float)(pl.org_d[q] + ((double)L.i[q] + (double)L.f[q]) * pl.vox_d[q]);
            a.ep_reason[slot] = escaped ? 1 : 0;
            break;
        }
        if (!SEC || traj >= nbr) break;
        // the next secondary: from its branch point, turned by its emission angles,
        // all of its steps whole
        {
            const Branch B = br[traj++];
            const DevSec sc = a.secs[B.j];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                L.i[q] = B.i[q];
                L.f[q] = B.f[q];
                L.b[q] = B.b[q];
            }
            turn_direction(L.b, sc.st, sc.ct, sc.cph, sc.sph);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                L.d[q] = LISTED ? lm[3 * q + 0] * L.b[0] + lm[3 * q + 1] * L.b[1] + lm[3 * q + 2] * L.b[2]
                                : wc[3 * q + 0] * L.b[0] + wc[3 * q + 1] * L.b[1] + wc[3 * q + 2] * L.b[2];
            {
                const float iv[3] = {wc[9], wc[10], wc[11]};
                set_direction_terms(L.d, iv, ta, tb, dv);
            }
            L.v = ((uint32_t)L.i[2] * (uint32_t)ny + (uint32_t)L.i[1]) * (uint32_t)nx + (uint32_t)L.i[0];
            k = sc.k0;
            kend = sc.k1;
            tau0 = 0.0;
            g20 = 0.0;
        }
    }
    esc = I_h - hdep;                               // escaped, or deposited upstream (up), or 0
}

// a value the same in every lane, as the first active lane's (so the compiler
// keeps it in a scalar register)
__device__ inline float uniform_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

__device__ inline long long wave_sum(long long x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

template <bool EP, bool SEC, bool CNT, class Sink>
__device__ void process_unit(const TransportArgs &a, const float2 *lut, unsigned long long unit,
                             uint32_t lane, const Sink &sink)
{
    // the work item holding this unit: largest i with items[i].unit0 <= unit
    uint32_t lo = 0, hi = a.n_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.items[mid].unit0 <= unit) lo = mid; else hi = mid;
    }
    const WorkItem it = a.items[lo];
    const DevSpot &sp = a.spots[it.gspot];
    const DevPlan &pl = a.plans[sp.plan];
    const unsigned long long h0 = it.h0 + (a.hnext ? a.hnext[it.gspot] : 0ull);
    // the lane's history: consecutive (a 64-aligned chunk sharing a track), or
    // the run's order by start position
    unsigned long long h;
    bool valid;
    if (a.order) {
        const uint32_t off = a.order[unit * kWave + lane];
        h = h0 + off;
        valid = off != 0xFFFFFFFFu;
    } else {
        h = (h0 / kWave + (unit - it.unit0)) * kWave + lane;
        valid = h >= h0 && h < h0 + it.n;
    }
    long long inc = 0, esc = 0;
    WorkCount wk{0u, 0u, 0u};
    // the wave's constants (a unit is one source's: the same in every lane)
    float wc[12];
#pragma unroll
    for (int q = 0; q < 9; ++q) wc[q] = uniform_f(sp.m[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q) wc[9 + q] = uniform_f(pl.inv_vox[q]);
    if (valid) {
        if (sp.kind)                                  // (wave-uniform: a unit is one source's)
            replay_history<EP, true, SEC, CNT>(a, sp, pl, lut, wc, h, (uint32_t)(h - h0), inc, esc, sink, wk);
        else
            replay_history<EP, false, SEC, CNT>(a, sp, pl, lut, wc, h, (uint32_t)(h - h0), inc, esc, sink, wk);
    }
    if (!EP) {
        inc = wave_sum(inc);
        esc = wave_sum(esc);
        if (lane == 0) {
            if (inc) add_global(pl.acc + 0, (unsigned long long)inc);
            if (esc) add_global(pl.acc + 1, (unsigned long long)esc);
        }
        if (CNT) {                                    // the plan's work counters
            const long long ws = wave_sum((long long)wk.steps), wv = wave_sum((long long)wk.visits),
                            wf = wave_sum((long long)wk.flushes);
            if (lane == 0) {
                add_global(pl.acc + 4, (unsigned long long)ws);
                add_global(pl.acc + 5, (unsigned long long)wv);
                add_global(pl.acc + 6, (unsigned long long)wf);
            }
        }
    }
}

// the plan whose tallies a unit deposits into (the LDS sink needs it for its
// fallback and its flush)
__device__ inline const DevPlan *plan_of_unit(const TransportArgs &a, unsigned long long unit)
{
    uint32_t lo = 0, hi = a.n_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.items[mid].unit0 <= unit) lo = mid; else hi = mid;
    }
    return a.plans + a.spots[a.items[lo].gspot].plan;
}

__device__ inline unsigned long long scalar_u64(unsigned long long x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <bool VAR, bool EP, bool SEC, bool CNT = false>
__global__ void __launch_bounds__(1024) transport_kernel(TransportArgs a)
{
    __shared__ float2 s_lut[kLutSize];
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) s_lut[i] = a.lut[i];
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // scalar
    const uint32_t wpb = blockDim.x / kWave;
    if (a.queue == nullptr) {
        const unsigned long long unit = (unsigned long long)blockIdx.x * wpb + wave;
        if (unit < a.n_units) {
            if (EP) process_unit<EP, SEC, CNT>(a, s_lut, unit, lane, NullSink{});
            else {
                const DevPlan *pl = plan_of_unit(a, unit);
                process_unit<EP, SEC, CNT>(a, s_lut, unit, lane, GlobalSink<VAR>{pl->E, pl->E2});
            }
        }
        return;
    }
    // persistent: each wave pulls units from a global counter until none are
    // left.  Every lane executes the atomic (lane 0 adds 1, the others 0), so
    // there is no divergent branch around it, and lane 0's old value - a unique
    // ticket - is read back with readfirstlane as a scalar: the loop exit is a
    // uniform branch and no cross-lane read sits in divergent control flow.
    for (;;) {
        const unsigned long long unit = scalar_u64(atomicAdd(a.queue, lane == 0 ? 1ull : 0ull));
        if (unit >= a.n_units) break;
        if (EP) process_unit<EP, SEC, CNT>(a, s_lut, unit, lane, NullSink{});
        else {
            const DevPlan *pl = plan_of_unit(a, unit);
            process_unit<EP, SEC, CNT>(a, s_lut, unit, lane, GlobalSink<VAR>{pl->E, pl->E2});
        }
    }
}

// Persistent kernel with a per-workgroup LDS sub-tally.  The workgroup works in
// rounds: it claims wpb * upw consecutive units (wave w takes upw of them),
// every visit deposits into the LDS table, then after a barrier the table is
// flushed into the plans' tallies with one global atomic per occupied slot and
// cleared.  Units of one round come from the same spot or a neighbouring one,
// whose histories overlap in space, so most visits of a round merge in LDS.
// CACHE selects the sub-tally: the hash table with global fallback (LdsSink)
// or the write-back cache (CacheSink).
template <bool VAR, bool CACHE, bool SEC>
__global__ void __launch_bounds__(1024) transport_lds_kernel(TransportArgs a, uint32_t slots, uint32_t upw)
{
    __shared__ float2 s_lut[kLutSize];
    __shared__ unsigned long long s_claim;
    extern __shared__ unsigned long long s_dyn[];
    unsigned long long *s_e = s_dyn;
    unsigned long long *s_e2 = s_dyn + slots;
    uint32_t *s_key = (uint32_t *)(s_dyn + (VAR ? 2 : 1) * slots);
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) s_lut[i] = a.lut[i];
    for (uint32_t i = threadIdx.x; i < slots; i += blockDim.x) {
        if (!CACHE) s_key[i] = kEmpty;
        s_e[i] = 0;
        if (VAR) s_e2[i] = 0;
    }
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // scalar
    const uint32_t wpb = blockDim.x / kWave;
    const unsigned long long per_round = (unsigned long long)wpb * upw;
    for (;;) {
        // one ticket per round for the whole workgroup, taken by thread 0's
        // lane of the atomic (every lane executes it, the others add 0)
        const unsigned long long got = atomicAdd(a.queue, threadIdx.x == 0 ? per_round : 0ull);
        if (threadIdx.x == 0) s_claim = got;
        __syncthreads();
        const unsigned long long base = scalar_u64(s_claim);
        if (base >= a.n_units) break;
        const DevPlan *tab_pl = plan_of_unit(a, base);
        // value bits of a cache word: the key needs bit_width(voxel count)
        const uint32_t nvox = (uint32_t)tab_pl->n[0] * (uint32_t)tab_pl->n[1] * (uint32_t)tab_pl->n[2];
        const uint32_t vbits = 64u - (32u - (uint32_t)__builtin_clz(nvox | 1u));
        for (uint32_t j = 0; j < upw; ++j) {
            const unsigned long long unit = base + (unsigned long long)wave * upw + j;
            if (unit >= a.n_units) break;
            const DevPlan *pl = plan_of_unit(a, unit);
            if (CACHE)
                process_unit<false, SEC, false>(a, s_lut, unit, lane,
                                         CacheSink<VAR>{pl->E, pl->E2, pl == tab_pl, s_e, s_e2, slots, vbits, nvox});
            else
                process_unit<false, SEC, false>(a, s_lut, unit, lane,
                                         LdsSink<VAR>{pl->E, pl->E2, pl == tab_pl, s_key, s_e, s_e2, slots - 1});
        }
        __syncthreads();
        // flush: one atomic per occupied slot; consecutive slots often hold
        // consecutive voxels, so neighbouring lanes' atomics share lines
        unsigned long long *const tE = tab_pl->E, *const tE2 = tab_pl->E2;
        for (uint32_t i = threadIdx.x; i < slots; i += blockDim.x) {
            if (CACHE) {
                const CacheSink<VAR> cs{tE, tE2, true, s_e, s_e2, slots, vbits, nvox};
                const unsigned long long w = s_e[i];
                if (w) {
                    cs.flush_word(tE, w);
                    s_e[i] = 0;
                }
                if (VAR) {
                    const unsigned long long w2 = s_e2[i];
                    if (w2) {
                        cs.flush_word(tE2, w2);
                        s_e2[i] = 0;
                    }
                }
            } else {
                const uint32_t k = s_key[i];
                if (k != kEmpty) {
                    const unsigned long long ev = s_e[i];
                    if (ev) add_global(tE + k, ev);
                    if (VAR) {
                        const unsigned long long e2v = s_e2[i];
                        if (e2v) add_global(tE2 + k, e2v);
                        s_e2[i] = 0;
                    }
                    s_e[i] = 0;
                    s_key[i] = kEmpty;
                }
            }
        }
        __syncthreads();
    }
}

// Persistent kernel with a whole-launch LDS write-back cache, for launches of
// one plan: no rounds and no barriers between units, evictions reach HBM as
// they happen, and the workgroup flushes the cache once when the queue is
// empty.  The workgroup takes units from the global queue in chunks of
// `chunk` consecutive units (histories of one spot, which overlap in space)
// and its waves take units of the current chunk one by one, so the waves
// sharing the cache work on neighbouring histories.  The chunk word in LDS is
// (first unit << 16 | units handed out); the wave that draws index `chunk`
// fetches the next chunk, waves that draw past it wait until the word holds
// a new chunk (that wave's fetch never waits on anything).
template <bool VAR, bool SEC>
__global__ void __launch_bounds__(1024) transport_cache_kernel(TransportArgs a, uint32_t slots, uint32_t chunk)
{
    __shared__ float2 s_lut[kLutSize];
    __shared__ unsigned long long s_chunk;
    extern __shared__ unsigned long long s_dyn[];
    unsigned long long *s_e = s_dyn;
    unsigned long long *s_e2 = s_dyn + slots;
    for (int i = threadIdx.x; i < kLutSize; i += blockDim.x) s_lut[i] = a.lut[i];
    for (uint32_t i = threadIdx.x; i < slots; i += blockDim.x) {
        s_e[i] = 0;
        if (VAR) s_e2[i] = 0;
    }
    const unsigned long long n_units = a.n_units;
    // the first chunk (a start at or past the end means no work)
    const unsigned long long first = atomicAdd(a.queue, threadIdx.x == 0 ? (unsigned long long)chunk : 0ull);
    if (threadIdx.x == 0) s_chunk = (first < n_units ? first : n_units) << 16;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // scalar
    const DevPlan *pl = plan_of_unit(a, 0);                   // the launch's one plan
    const uint32_t nvox = (uint32_t)pl->n[0] * (uint32_t)pl->n[1] * (uint32_t)pl->n[2];
    const uint32_t vbits = 64u - (32u - (uint32_t)__builtin_clz(nvox | 1u));
    unsigned long long *const E = pl->E, *const E2 = pl->E2;
    const CacheSink<VAR> cs{E, E2, true, s_e, s_e2, slots, vbits, nvox};
    volatile unsigned long long *const chunk_word = &s_chunk;
    for (;;) {
        // every lane executes the LDS atomic (lane 0 adds 1), lane 0's old value is the ticket
        const unsigned long long w = scalar_u64(atomicAdd(&s_chunk, lane == 0 ? 1ull : 0ull));
        const unsigned long long base = w >> 16;
        const uint32_t idx = (uint32_t)(w & 0xffffu);
        if (base >= n_units) break;
        if (idx < chunk) {
            const unsigned long long unit = base + idx;
            if (unit < n_units) process_unit<false, SEC, false>(a, s_lut, unit, lane, cs);
        } else if (idx == chunk) {
            const unsigned long long nb = scalar_u64(atomicAdd(a.queue, lane == 0 ? (unsigned long long)chunk : 0ull));
            if (lane == 0) atomicExch(&s_chunk, (nb < n_units ? nb : n_units) << 16);
        } else {
            // the wave that drew `chunk` replaces the word with a later chunk (or the end)
            while ((scalar_u64(*chunk_word) >> 16) == base) __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < slots; i += blockDim.x) {
        cs.flush_word(E, s_e[i]);
        if (VAR) cs.flush_word(E2, s_e2[i]);
    }
}

template <bool SEC>
hipError_t launch_transport_t(const TransportArgs &a, dim3 grid, dim3 block, bool variance, bool endpoints,
                              bool count, hipStream_t s)
{
    if (count && variance)
        hipLaunchKernelGGL((transport_kernel<true, false, SEC, true>), grid, block, 0, s, a);
    else if (count)
        hipLaunchKernelGGL((transport_kernel<false, false, SEC, true>), grid, block, 0, s, a);
    else if (endpoints)
        hipLaunchKernelGGL((transport_kernel<false, true, SEC>), grid, block, 0, s, a);
    else if (variance)
        hipLaunchKernelGGL((transport_kernel<true, false, SEC>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((transport_kernel<false, false, SEC>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <bool SEC>
hipError_t launch_transport_lds_t(const TransportArgs &a, dim3 grid, dim3 block, size_t dyn, uint32_t slots,
                                  uint32_t units_per_wave, uint32_t waves_per_block, bool variance, uint32_t mode,
                                  hipStream_t s)
{
    if (mode == 2 && variance)
        hipLaunchKernelGGL((transport_cache_kernel<true, SEC>), grid, block, dyn, s, a, slots, waves_per_block * units_per_wave);
    else if (mode == 2)
        hipLaunchKernelGGL((transport_cache_kernel<false, SEC>), grid, block, dyn, s, a, slots, waves_per_block * units_per_wave);
    else if (mode && variance)
        hipLaunchKernelGGL((transport_lds_kernel<true, true, SEC>), grid, block, dyn, s, a, slots, units_per_wave);
    else if (mode)
        hipLaunchKernelGGL((transport_lds_kernel<false, true, SEC>), grid, block, dyn, s, a, slots, units_per_wave);
    else if (variance)
        hipLaunchKernelGGL((transport_lds_kernel<true, false, SEC>), grid, block, dyn, s, a, slots, units_per_wave);
    else
        hipLaunchKernelGGL((transport_lds_kernel<false, false, SEC>), grid, block, dyn, s, a, slots, units_per_wave);
    return hipGetLastError();
}

} // namespace

hipError_t launch_transport(const TransportArgs &a, uint32_t waves_per_block, uint32_t grid_blocks,
                            bool variance, bool endpoints, hipStream_t s, bool count)
{
    const dim3 block(waves_per_block * kWave);
    const dim3 grid(grid_blocks);
    return a.secs ? launch_transport_t<true>(a, grid, block, variance, endpoints, count, s)
                  : launch_transport_t<false>(a, grid, block, variance, endpoints, count, s);
}

size_t lds_tally_bytes(uint32_t slots, bool variance, uint32_t mode)
{
    return (size_t)slots * ((variance ? 16 : 8) + (mode ? 0 : 4));
}

hipError_t prepare_lds_kernels()
{
    const int dyn = (int)(kMaxLdsBytes - kLutSize * sizeof(float2) - kLdsFixedBytes);
    const void *k[12] = {(const void *)transport_lds_kernel<true, false, false>,
                         (const void *)transport_lds_kernel<false, false, false>,
                         (const void *)transport_lds_kernel<true, true, false>,
                         (const void *)transport_lds_kernel<false, true, false>,
                         (const void *)transport_cache_kernel<true, false>, (const void *)transport_cache_kernel<false, false>,
                         (const void *)transport_lds_kernel<true, false, true>,
                         (const void *)transport_lds_kernel<false, false, true>,
                         (const void *)transport_lds_kernel<true, true, true>,
                         (const void *)transport_lds_kernel<false, true, true>,
                         (const void *)transport_cache_kernel<true, true>, (const void *)transport_cache_kernel<false, true>};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 12 && e == hipSuccess; ++i)
        e = hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    return e;
}

// Workgroups of the whole-launch cache kernel (waves_per_block waves, `slots`
// LDS slots per tally) that fit one CU at once.  The kernel's waves wait on an
// LDS word that a sibling wave of the same workgroup writes; a workgroup is
// dispatched whole, so its waves are resident together whenever it runs at
// all, and this is at least 1 exactly when the launch can run.
hipError_t cache_kernel_occupancy(uint32_t waves_per_block, uint32_t slots, bool variance, int *blocks)
{
    // (the kernels with and without secondaries: the launch may use either)
    const void *k[2] = {variance ? (const void *)transport_cache_kernel<true, false>
                                 : (const void *)transport_cache_kernel<false, false>,
                        variance ? (const void *)transport_cache_kernel<true, true>
                                 : (const void *)transport_cache_kernel<false, true>};
    int b[2] = {0, 0};
    for (int i = 0; i < 2; ++i) {
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(b + i, k[i], (int)(waves_per_block * kWave),
                                                                          lds_tally_bytes(slots, variance, 2));
        if (e != hipSuccess) return e;
    }
    *blocks = b[0] < b[1] ? b[0] : b[1];
    return hipSuccess;
}

hipError_t launch_transport_lds(const TransportArgs &a, uint32_t waves_per_block, uint32_t grid_blocks,
                                uint32_t slots, uint32_t units_per_wave, bool variance, uint32_t mode, hipStream_t s)
{
    const dim3 block(waves_per_block * kWave);
    const dim3 grid(grid_blocks);
    const size_t dyn = lds_tally_bytes(slots, variance, mode);
    return a.secs ? launch_transport_lds_t<true>(a, grid, block, dyn, slots, units_per_wave, waves_per_block, variance,
                                                 mode, s)
                  : launch_transport_lds_t<false>(a, grid, block, dyn, slots, units_per_wave, waves_per_block, variance,
                                                  mode, s);
}

} // namespace fdc
