/*
 * CPU oracle for track-repeating proton dose calculation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the HIP path (no headers, tables or helpers); both read the same
 * seeded inputs.
 *
 * Plain and slow on purpose: FP64 geometry, absolute positions, one history at
 * a time, integer fixed-point tallies (1 LSB = 2^-24 MeV).  It follows the two
 * tasks of the GPU kernel in Section 2.3 of the paper:
 *   task 1 - find the database history, select the trajectory and the start step;
 *   task 2 - re-trace the stored water steps through the voxel phantom, scaling
 *            each step's length and scattering angle by the local material
 *            (Section 2.2), and tally the deposited energy (Section 2.3).
 * Where the paper is silent the readings below fix the behaviour:
 *   - a step keeps its energy loss; its water-equivalent length (WEL) is
 *     consumed voxel by voxel, geometric length = WEL / RSP;
 *   - energy is deposited uniformly in WEL along a step, split with a
 *     telescoping round-to-nearest-even so the pieces sum exactly;
 *   - the deflection is applied at the end of a step (condensed history,
 *     Section 2.1) with angle theta * sqrt(sum(w_v * G_v) / WEL), G = RScP/RSP;
 *   - the direction lives in the beam frame and is rotated with the textbook
 *     polar/azimuth formula, then mapped by the field matrix M = [e1 e2 d];
 *   - histories of one spot come in chunks of R consecutive indices sharing one
 *     database track (the paper feeds one history to a whole thread group,
 *     Section 4); every random number is Philox4x32-10 keyed by the run seed
 *     with a counter made of the history identity;
 *   - voxels with HU below the vacuum threshold are free flight;
 *   - leaving the phantom box ends the history; its undeposited energy is
 *     counted as escaped.
 *   - per-history per-voxel-visit deposits are squared for the sum-of-squares
 *     tally used by the history-by-history uncertainty, Eq. (2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FP_SCALE 16777216.0 /* 2^24 LSB per MeV */
#define TAG_TRACK 2u
#define TAG_SRC 3u
#define FLAG_VARIANCE 1u
#define FLAG_ROTATE 2u

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11.  Ten rounds of the 4x32 S-box with key bump. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u; /* golden ratio */
            k1 += 0xBB67AE85u; /* sqrt(3) - 1 */
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* n counters ctr[4n] under one key, into out[4n] */
void oracle_philox_batch(const uint32_t *ctr, const uint32_t key[2], uint32_t *out, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* uniform in the open interval (0,1): 24 high bits plus half an LSB */
double oracle_uniform(uint32_t x)
{
    return (double)(x >> 8) * (1.0 / 16777216.0) + (1.0 / 33554432.0);
}

/* ---------------------------------------------------------------------- */
/* HU -> material, piecewise linear over the table points, clamped at the ends */
typedef struct {
    const double *hu, *rho, *rsp, *rscp;
    int n;
    double vacuum_below_hu;
} hu_table;

static double interp(const hu_table *t, const double *val, double h)
{
    if (h <= t->hu[0]) return val[0];
    if (h >= t->hu[t->n - 1]) return val[t->n - 1];
    int j = 0;
    while (!(h < t->hu[j + 1])) ++j;
    return val[j] + (val[j + 1] - val[j]) * (h - t->hu[j]) / (t->hu[j + 1] - t->hu[j]);
}

/* HU value after clamping to the CT range [-1024, 3071] */
static double clamp_hu(int16_t v)
{
    int h = v;
    if (h < -1024) h = -1024;
    if (h > 3071) h = 3071;
    return (double)h;
}

/* material of a voxel: is it vacuum, its RSP and G = RScP/RSP */
static int material(const hu_table *t, int16_t v, double *rsp, double *g)
{
    double h = clamp_hu(v);
    if (h < t->vacuum_below_hu) { *rsp = 0.0; *g = 0.0; return 1; }
    double s = interp(t, t->rsp, h);
    double c = interp(t, t->rscp, h);
    *rsp = s;
    *g = s > 0.0 ? c / s : 0.0;
    return s <= 0.0;
}

void oracle_material(const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                     int n_pts, double vacuum_below_hu, const int16_t *hu_in, int n,
                     double *rho_out, double *rsp_out, double *g_out, uint8_t *vac_out)
{
    hu_table t = {hu_pts, rho, rsp, rscp, n_pts, vacuum_below_hu};
    for (int i = 0; i < n; ++i) {
        double s, g;
        vac_out[i] = (uint8_t)material(&t, hu_in[i], &s, &g);
        rsp_out[i] = s;
        g_out[i] = g;
        rho_out[i] = interp(&t, t.rho, clamp_hu(hu_in[i]));
    }
}

/* ---------------------------------------------------------------------- */
/* Optional record of one history's walk (test aid): one event per voxel
 * visit and per step end, in the order they happen. */
typedef struct {
    int64_t *ev;  /* per event: kind, voxel index, deposited piece (fp), exit axis (-1: none) */
    double *evd;  /* per event: WEL consumed, geometric length moved */
    int cap, n;
} oracle_trace;

enum { EV_VOXEL = 0, EV_VACUUM = 1, EV_STEP_END = 2, EV_ESCAPE = 3 };

static void trace_push(oracle_trace *tr, int64_t kind, int64_t v, int64_t piece, int64_t axis, double w,
                       double move)
{
    if (!tr) return;
    if (tr->n < tr->cap) {
        int64_t *e = tr->ev + 4 * tr->n;
        e[0] = kind; e[1] = v; e[2] = piece; e[3] = axis;
        tr->evd[2 * tr->n] = w;
        tr->evd[2 * tr->n + 1] = move;
    }
    tr->n++;
}

typedef struct {
    /* track database */
    const float *steps; /* 4 floats per step: dx (WEL cm), dE (MeV), theta, phi */
    const uint64_t *track_off;
    uint32_t n_tracks;
    const float *bin_E;
    const uint32_t *bin_first;
    uint32_t n_bins;
    /* phantom */
    const int16_t *hu;
    int n[3];
    double vox[3], org[3];
    hu_table tab;
    /* spots */
    const float *spot_pos, *spot_dir, *spot_E, *spot_sigma;
    /* sources read from a phase-space list instead (Section 2.3: incident
     * protons read from a file): source s with ps_count[s] > 0 is the protons
     * ps_first[s] .. ps_first[s] + ps_count[s] - 1, each with its own position,
     * direction and energy; history h of it is proton ps_first[s] + h mod
     * ps_count[s] (a new pass over the list re-uses it with new tracks).
     * NULL: every source is a spot. */
    const uint64_t *ps_first, *ps_count;
    const float *ps_pos, *ps_dir, *ps_E;
    /* beam-line devices upstream of the phantom (an aperture and a range
     * compensator on one pixel grid; the GPU code of the paper had none,
     * Section 4): spot s passes device spot_dev[s] (-1: none).  Device i:
     * dev_par[16 i ..] = upstream-face centre (3), face normal along the beam
     * (3), pixel pitch along the normal's lateral axes e1, e2 (2), pixels
     * along e1, e2 (2), compensator RSP and RScP (2); its pixels (e1 fastest)
     * are dev_pix[dev_pix_off[i] ..]: < 0 closed, else the compensator
     * thickness (cm, along the normal).  NULL: no devices. */
    const int32_t *spot_dev;
    const double *dev_par;
    const float *dev_pix;
    const uint64_t *dev_pix_off;
    /* secondary trajectories of the database (NULL sec_first: none): track t
     * has secondaries sec_first[t] .. sec_first[t+1]-1; secondary j starts at
     * the end of the track's primary step sec_branch[j] (counted from its first
     * step), leaves at polar angle sec_emit[2j] and azimuth sec_emit[2j+1]
     * from the primary's direction there, and has steps sec_steps[4 sec_off[j]
     * ..] up to sec_off[j+1] (4 floats each, as the primary's). */
    const uint32_t *sec_first, *sec_branch;
    const uint64_t *sec_off;
    const float *sec_steps, *sec_emit;
    /* run */
    uint32_t plan;
    uint64_t seed;
    uint32_t R;
    uint32_t flags;
    oracle_trace *trace; /* NULL unless a test asks for the walk */
} oracle_problem;

typedef struct {
    int64_t *E;
    uint64_t *E2;
    int64_t incident, escaped;
    uint64_t steps, visits, vacuum_visits, flushes;
    /* optional: the squared-energy tally of Eq. (2) taken literally - the
     * square of a history's whole deposit in a voxel, summed over every visit
     * of that history (E2 squares each visit on its own) */
    uint64_t *E2x;
    int64_t *hsum;      /* per voxel: this history's deposit so far */
    size_t *touched;    /* voxels with a non-zero hsum */
    size_t n_touched, cap_touched;
    int overflow;
} oracle_tally;

static int64_t fp_energy(double e) { return (int64_t)nearbyint(e * FP_SCALE); }

/* right-handed lateral axes of a beam direction: d = +z gives (x, y) */
static void field_frame(const double d[3], double e1[3], double e2[3])
{
    double a[3] = {0.0, 0.0, 1.0};
    if (fabs(d[2]) >= 0.9) { a[0] = 1.0; a[2] = 0.0; }
    e2[0] = d[1] * a[2] - d[2] * a[1];
    e2[1] = d[2] * a[0] - d[0] * a[2];
    e2[2] = d[0] * a[1] - d[1] * a[0];
    double l = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    e2[0] /= l; e2[1] /= l; e2[2] /= l;
    e1[0] = e2[1] * d[2] - e2[2] * d[1];
    e1[1] = e2[2] * d[0] - e2[0] * d[2];
    e1[2] = e2[0] * d[1] - e2[1] * d[0];
}

/* polar/azimuth rotation of a unit direction (u,v,w) by (theta, phi) */
static void rotate(double dir[3], double theta, double phi)
{
    double u = dir[0], v = dir[1], w = dir[2];
    double ct = cos(theta), st = sin(theta), cp = cos(phi), sp = sin(phi);
    double rho = hypot(u, v);
    double nu, nv, nw;
    if (rho < 1e-20) {
        nu = st * cp;
        nv = st * sp;
        nw = (w < 0.0 ? -1.0 : 1.0) * ct;
    } else {
        nu = u * ct + st * (u * w * cp - v * sp) / rho;
        nv = v * ct + st * (v * w * cp + u * sp) / rho;
        nw = w * ct - rho * st * cp;
    }
    double l = sqrt(nu * nu + nv * nv + nw * nw);
    dir[0] = nu / l; dir[1] = nv / l; dir[2] = nw / l;
}

void oracle_rotate(double dir[3], double theta, double phi) { rotate(dir, theta, phi); }

static void flush(const oracle_problem *P, oracle_tally *T, size_t v, int64_t *acc)
{
    if (*acc == 0) return;
    if (T->E2x) {
        if (T->hsum[v] == 0) {
            if (T->n_touched < T->cap_touched) T->touched[T->n_touched++] = v;
            else T->overflow = 1;
        }
        T->hsum[v] += *acc;
    }
    T->E[v] += *acc;
    if ((P->flags & FLAG_VARIANCE) && T->E2) {
        uint64_t q = (uint64_t)((*acc + 2048) >> 12);
        T->E2[v] += q * q;
    }
    T->flushes++;
    *acc = 0;
}

enum { END_STOP = 0, END_ESCAPE = 1, END_MISS = 2, END_UPSTREAM = 3 };

/* Step k of the track as replayed: water-equivalent length, energy (fixed
 * point), polar and azimuthal deflection.  The first replayed step k0 is the
 * part of step k0 left below the spot energy (fraction f of its energy):
 * length f dx, angle theta sqrt(f) (Highland's sqrt of the length), azimuth
 * turned by phi0 (track rotation). */
static void step_params(const float *st, uint64_t k, uint64_t k0, int64_t cum, int64_t skip, double phi0,
                        double *w_tot, int64_t *e, double *theta, double *phi)
{
    *w_tot = st[4 * k + 0];
    *theta = st[4 * k + 2];
    *phi = st[4 * k + 3];
    *e = fp_energy(st[4 * k + 1]);
    if (k == k0) {
        int64_t e_first = cum + *e - skip;
        double f = (double)e_first / (double)*e;
        *e = e_first;
        *w_tot *= f;
        *theta *= sqrt(f);
        *phi += phi0;
    }
}

/* Where a history stands when it reaches the phantom: the step being
 * replayed and how much of it is done (WEL consumed, energy deposited so far
 * in fixed point, sum of w G), its beam-frame direction, and the energy
 * deposited upstream of the phantom. */
typedef struct {
    uint64_t k;
    double tau, g2;
    int64_t dep;
    double db[3];
    int64_t up_dep;
} replay_state;

/* The beam-line device dv (see oracle_problem) on the history's way: the ray
 * from pos along d meets the device's upstream face at one pixel; a closed
 * pixel, a pixel off the grid, or a face not ahead of the start point
 * (direction not towards it) stops the history there.  An open pixel with a
 * compensator thickness T > 0: the track is replayed through a slab of the
 * compensator's material from that point until the displacement along the
 * normal reaches T - each step's WEL consumed at geometric length WEL / RSP,
 * its energy split uniformly in WEL with the telescoping rounding, the
 * deflection at the step end scaled by sqrt(sum w G / WEL) with G = RScP/RSP,
 * as in a voxel (the slab's thickness is the one of the pixel it was entered
 * through).  The energy deposited there is absorbed upstream.  Returns 1 if
 * the history ends on or in the device (blocked, or its track ends in the
 * compensator), else 0 with pos, d and the state at the exit face. */
static int device_pass(const oracle_problem *P, int dv, const float *st, uint64_t n_steps, uint64_t k0,
                       int64_t cum, int64_t skip, double phi0, double M[3][3], double pos[3], double d[3],
                       replay_state *S)
{
    const double *q = P->dev_par + 16 * dv;
    double o[3] = {q[0], q[1], q[2]}, nrm[3] = {q[3], q[4], q[5]};
    double nl = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    for (int a = 0; a < 3; ++a) nrm[a] /= nl;
    double u1[3], u2[3];
    field_frame(nrm, u1, u2);
    const long n0 = (long)q[8], n1 = (long)q[9];
    const double rsp = q[10], g = q[11] / q[10];
    double dn = d[0] * nrm[0] + d[1] * nrm[1] + d[2] * nrm[2];
    double t = ((o[0] - pos[0]) * nrm[0] + (o[1] - pos[1]) * nrm[1] + (o[2] - pos[2]) * nrm[2]);
    if (!(dn > 0.0) || t < 0.0) return 1;
    t /= dn;
    for (int a = 0; a < 3; ++a) pos[a] += t * d[a];
    double ra = 0.0, rb = 0.0;
    for (int a = 0; a < 3; ++a) {
        ra += (pos[a] - o[a]) * u1[a];
        rb += (pos[a] - o[a]) * u2[a];
    }
    double fi = floor(ra / q[6] + 0.5 * (double)n0), fj = floor(rb / q[7] + 0.5 * (double)n1);
    if (fi < 0.0 || fj < 0.0 || fi >= (double)n0 || fj >= (double)n1) return 1;
    double thick = P->dev_pix[P->dev_pix_off[dv] + (uint64_t)fj * (uint64_t)n0 + (uint64_t)fi];
    if (thick < 0.0) return 1;
    if (thick == 0.0) return 0;
    double z = 0.0; /* displacement along the normal inside the slab */
    for (uint64_t k = k0; k < n_steps; ++k) {
        double w_tot, theta, phi;
        int64_t e;
        step_params(st, k, k0, cum, skip, phi0, &w_tot, &e, &theta, &phi);
        double tau = 0.0, g2 = 0.0;
        int64_t dep = 0;
        int on_face = 0;            /* the step ended exactly on the exit face */
        while (tau < w_tot) {
            dn = d[0] * nrm[0] + d[1] * nrm[1] + d[2] * nrm[2];
            double lgeo = dn > 0.0 ? (thick - z) / dn : INFINITY;
            if (lgeo < 0.0) lgeo = 0.0;
            double rem = w_tot - tau, wb = lgeo * rsp, w_v, tau_n, move;
            int exits;
            if (rem <= wb) { /* the step ends in the slab (or on its exit face) */
                w_v = rem;
                tau_n = w_tot;
                move = rem / rsp;
                exits = (rem == wb);
            } else {
                w_v = wb;
                tau_n = tau + wb;
                move = lgeo;
                exits = 1;
            }
            int64_t cumk = (int64_t)nearbyint((double)e * (tau_n / w_tot));
            if (tau_n >= w_tot) cumk = e;
            S->up_dep += cumk - dep;
            dep = cumk;
            g2 += w_v * g;
            tau = tau_n;
            for (int a = 0; a < 3; ++a) pos[a] += move * d[a];
            z += move * dn;
            if (exits && tau < w_tot) { /* out through the exit face inside the step */
                S->k = k;
                S->tau = tau;
                S->g2 = g2;
                S->dep = dep;
                return 0;
            }
            on_face = exits;
        }
        /* deflection at the end of the step; a step ending exactly on the exit
         * face ends in the slab and the next one starts beyond it */
        rotate(S->db, theta * sqrt(g2 / w_tot), phi);
        for (int a = 0; a < 3; ++a) d[a] = M[a][0] * S->db[0] + M[a][1] * S->db[1] + M[a][2] * S->db[2];
        if (on_face) {
            S->k = k + 1;
            S->tau = 0.0;
            S->g2 = 0.0;
            S->dep = 0;
            return S->k >= n_steps;
        }
    }
    return 1; /* the track ended in the compensator */
}

/* Branch points of a track's secondary trajectories met by the primary's
 * walk (position, voxel, beam-frame direction at the end of the branch step). */
#define MAX_BRANCH 16
typedef struct {
    const uint32_t *branch;   /* branch step of each secondary of the track */
    uint32_t j, end;          /* next secondary to meet, one past the track's last */
    int n;
    uint32_t sec[MAX_BRANCH];
    double pos[MAX_BRANCH][3], db[MAX_BRANCH][3];
    int iv[MAX_BRANCH][3];
} branch_log;

/* Re-trace a trajectory's steps from k (its state: position, voxel, direction
 * d = M db, and for the first step replayed the part of it already done, tau0
 * WEL, dep0 energy, g20 sum w G) to n_steps: each step's WEL consumed voxel by
 * voxel at geometric length WEL / RSP, its energy split uniformly in WEL with
 * a telescoping round to nearest, the deflection at the step end scaled by
 * sqrt(sum w G / WEL) (Section 2.2); deposits flushed per voxel visit.
 * Steps k0 and beyond follow step_params (k0 the primary's partial first step;
 * a secondary passes k0 = UINT64_MAX).  With a branch log, the secondaries
 * starting at the end of a step are recorded there.  Adds the deposited
 * energy to *dep; returns END_STOP or END_ESCAPE (the remaining energy,
 * e_left minus what was deposited, goes to the trace's escape event). */
static int walk_trajectory(const oracle_problem *P, oracle_tally *T, const float *st, uint64_t k, uint64_t n_steps,
                           uint64_t k0, int64_t cum, int64_t skip, double phi0, double pos[3], int iv[3],
                           double d[3], double db[3], double M[3][3], double tau0, double g20, int64_t dep0,
                           branch_log *br, int64_t e_left, int64_t *hist_dep_out)
{
    int64_t acc = 0, hist_dep = 0;
    int reason = END_STOP;
    int alive = 1;
    const uint64_t k_begin = k;
    for (; k < n_steps && alive; ++k) {
        double w_tot, theta, phi;
        int64_t e;
        step_params(st, k, k0, cum, skip, phi0, &w_tot, &e, &theta, &phi);
        if (T) T->steps++;
        /* a step begun upstream (in a compensator) continues where it left off */
        double tau = k == k_begin ? tau0 : 0.0, g2 = k == k_begin ? g20 : 0.0;
        int64_t dep = k == k_begin ? dep0 : 0;
        while (tau < w_tot) {
            size_t v = ((size_t)iv[2] * P->n[1] + iv[1]) * P->n[0] + iv[0];
            double rsp, g;
            int vac = material(&P->tab, P->hu[v], &rsp, &g);
            /* distance to the voxel exit, ties resolved x -> y -> z */
            double lexit = INFINITY;
            int ax = -1;
            for (int a = 0; a < 3; ++a) {
                double ta;
                if (d[a] > 0.0) ta = (P->org[a] + (iv[a] + 1) * P->vox[a] - pos[a]) / d[a];
                else if (d[a] < 0.0) ta = (P->org[a] + iv[a] * P->vox[a] - pos[a]) / d[a];
                else continue;
                if (ta < 0.0) ta = 0.0;
                if (ta < lexit) { lexit = ta; ax = a; }
            }
            int cross = 1;
            double move = lexit;
            double w_trace = 0.0;
            int64_t piece_trace = 0;
            if (vac) {
                if (T) T->vacuum_visits++;
            } else {
                if (T) T->visits++;
                double rem = w_tot - tau;
                double wb = lexit * rsp;
                double w_v, tau_n;
                if (rem <= wb) { /* the step ends in this voxel (or on its exit face) */
                    w_v = rem;
                    tau_n = w_tot;
                    move = rem / rsp;
                    cross = (rem == wb);
                } else {
                    w_v = wb;
                    tau_n = tau + wb;
                }
                int64_t cumk = (int64_t)nearbyint((double)e * (tau_n / w_tot));
                if (tau_n >= w_tot) cumk = e;
                int64_t piece = cumk - dep;
                dep = cumk;
                acc += piece;
                hist_dep += piece;
                g2 += w_v * g;
                tau = tau_n;
                w_trace = w_v;
                piece_trace = piece;
            }
            trace_push(P->trace, vac ? EV_VACUUM : EV_VOXEL, (int64_t)v, piece_trace, cross ? ax : -1, w_trace,
                       move);
            if (cross) {
                for (int a = 0; a < 3; ++a) pos[a] += move * d[a];
                pos[ax] = P->org[ax] + (iv[ax] + (d[ax] > 0.0 ? 1 : 0)) * P->vox[ax];
                if (T) flush(P, T, v, &acc);
                iv[ax] += d[ax] > 0.0 ? 1 : -1;
                if (iv[ax] < 0 || iv[ax] >= P->n[ax]) {
                    trace_push(P->trace, EV_ESCAPE, -1, e_left - hist_dep, ax, 0.0, 0.0);
                    reason = END_ESCAPE;
                    alive = 0;
                    break;
                }
            } else {
                for (int a = 0; a < 3; ++a) pos[a] += move * d[a];
            }
        }
        if (!alive) break;
        /* deflection at the end of the step, scaled by the traversed material */
        double th = theta * sqrt(g2 / w_tot);
        trace_push(P->trace, EV_STEP_END, (int64_t)k, 0, -1, g2, th);
        rotate(db, th, phi);
        for (int a = 0; a < 3; ++a) d[a] = M[a][0] * db[0] + M[a][1] * db[1] + M[a][2] * db[2];
        /* secondary trajectories that start here */
        while (br && br->j < br->end && br->branch[br->j] == k) {
            if (br->n < MAX_BRANCH) {
                br->sec[br->n] = br->j;
                memcpy(br->pos[br->n], pos, sizeof(double) * 3);
                memcpy(br->db[br->n], db, sizeof(double) * 3);
                memcpy(br->iv[br->n], iv, sizeof(int) * 3);
                br->n++;
            }
            br->j++;
        }
    }
    if (alive && T) {
        size_t v = ((size_t)iv[2] * P->n[1] + iv[1]) * P->n[0] + iv[0];
        flush(P, T, v, &acc);
    }
    *hist_dep_out += hist_dep;
    return reason;
}

/* total energy of a secondary trajectory, fixed point */
static int64_t sec_energy(const oracle_problem *P, uint32_t j)
{
    int64_t e = 0;
    for (uint64_t k = P->sec_off[j]; k < P->sec_off[j + 1]; ++k) e += fp_energy(P->sec_steps[4 * k + 1]);
    return e;
}

/* One history (plan, spot s, index h).  Returns the end reason of its primary
 * trajectory; the end point is written to endpoint[3].  Tallies go to T (may
 * be NULL for endpoints only). */
static int replay_history(const oracle_problem *P, uint32_t s, uint64_t h, oracle_tally *T,
                          double endpoint[3])
{
    const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};

    /* ---- task 1: database history, trajectory and start step ---------- */
    const int listed = P->ps_count && P->ps_count[s] > 0; /* a proton from the phase-space list */
    const uint64_t pi = listed ? P->ps_first[s] + h % P->ps_count[s] : 0;
    double E_spot = listed ? P->ps_E[pi] : P->spot_E[s];
    uint32_t b = 0;
    while (b < P->n_bins && (double)P->bin_E[b] < E_spot) ++b;
    if (b >= P->n_bins) { /* above the database's top bin: not a valid source */
        for (int a = 0; a < 3; ++a) endpoint[a] = 0.0;
        return -1;
    }
    uint32_t n_b = P->bin_first[b + 1] - P->bin_first[b];

    uint64_t c = h / P->R; /* chunk of R histories sharing one track */
    uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), s, (P->plan << 4) | TAG_TRACK};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    uint32_t t = P->bin_first[b] + (uint32_t)(((uint64_t)x[0] * n_b) >> 32);

    const float *st = P->steps + 4 * P->track_off[t];
    uint64_t n_steps = P->track_off[t + 1] - P->track_off[t];
    /* the track's secondary trajectories (Section 2.2), each starting at the
     * end of a primary step; their energy is part of the track's */
    const uint32_t j_begin = P->sec_first ? P->sec_first[t] : 0, j_end = P->sec_first ? P->sec_first[t + 1] : 0;

    /* energy skip of a spot below its bin energy, and the start step
     * (Section 2.3, task 1): the energy below the bin's goes in the order the
     * track spends it - each primary step's loss, then the secondaries that
     * start at its end.  A skip that ends inside a secondary's energy drops
     * that secondary and starts at the next primary step whole (the incident
     * energy is then the track's after it). */
    int64_t skip = fp_energy(P->bin_E[b]) - fp_energy(E_spot);
    int64_t T_fp = 0;
    for (uint64_t k = 0; k < n_steps; ++k) T_fp += fp_energy(st[4 * k + 1]);
    for (uint32_t j = j_begin; j < j_end; ++j) T_fp += sec_energy(P, j);
    uint64_t k0 = 0;
    int64_t cum = 0;
    uint32_t j_first = j_begin;
    while (k0 < n_steps) {
        int64_t e = fp_energy(st[4 * k0 + 1]);
        if (cum + e > skip) break;
        cum += e;
        while (j_first < j_end && P->sec_branch[j_first] == k0) cum += sec_energy(P, j_first++);
        ++k0;
        if (cum > skip) {
            skip = cum;
            break;
        }
    }
    int64_t I_h = T_fp - skip;
    if (I_h < 0) I_h = 0;
    int64_t E_sec = 0; /* energy of the secondaries still ahead */
    for (uint32_t j = j_first; j < j_end; ++j) E_sec += sec_energy(P, j);

    /* source: lateral position (Gaussian of standard deviation sigma, or for
     * sigma < 0 uniform over a disk of radius -sigma: the circular field of
     * Section 2.5), beam direction, optional track rotation */
    ctr[0] = (uint32_t)h; ctr[1] = (uint32_t)(h >> 32); ctr[2] = s;
    ctr[3] = (P->plan << 4) | TAG_SRC;
    oracle_philox4x32_10(ctr, key, x);
    /* a listed proton has no lateral spread: its own position and direction */
    double sig = listed ? 0.0 : P->spot_sigma[s];
    /* Gaussian: Box-Muller radius; disk: the radius whose square is uniform */
    double r = sig >= 0.0 ? sqrt(-2.0 * log(oracle_uniform(x[0]))) : sqrt(oracle_uniform(x[0]));
    double ang = 2.0 * M_PI * oracle_uniform(x[1]);
    double n1 = r * cos(ang), n2 = r * sin(ang);
    double phi0 = (P->flags & FLAG_ROTATE) ? 2.0 * M_PI * oracle_uniform(x[2]) : 0.0;

    const float *src_dir = listed ? P->ps_dir + 3 * pi : P->spot_dir + 3 * s;
    const float *src_pos = listed ? P->ps_pos + 3 * pi : P->spot_pos + 3 * s;
    double d[3] = {src_dir[0], src_dir[1], src_dir[2]};
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= dl; d[1] /= dl; d[2] /= dl;
    double e1[3], e2[3];
    field_frame(d, e1, e2);
    double M[3][3]; /* columns e1, e2, d */
    for (int a = 0; a < 3; ++a) { M[a][0] = e1[a]; M[a][1] = e2[a]; M[a][2] = d[a]; }
    double pos[3];
    for (int a = 0; a < 3; ++a)
        pos[a] = (double)src_pos[a] + fabs(sig) * (n1 * e1[a] + n2 * e2[a]);

    if (T) T->incident += I_h;

    /* a beam-line device on the way (aperture, range compensator) */
    replay_state S = {k0, 0.0, 0.0, 0, {0.0, 0.0, 1.0}, 0};
    const int dv = P->spot_dev ? P->spot_dev[s] : -1;
    if (dv >= 0 && I_h > 0 && device_pass(P, dv, st, n_steps, k0, cum, skip, phi0, M, pos, d, &S)) {
        memcpy(endpoint, pos, sizeof(double) * 3);
        if (T) T->escaped += I_h;
        return END_UPSTREAM;
    }

    /* ray-box entry; the region outside the box is vacuum */
    double tin = -INFINITY, tout = INFINITY;
    int ax_in = -1;
    for (int a = 0; a < 3; ++a) {
        double lo = P->org[a], hi = P->org[a] + P->n[a] * P->vox[a];
        if (d[a] == 0.0) {
            if (pos[a] < lo || pos[a] >= hi) { tin = INFINITY; break; }
        } else {
            double t1 = (lo - pos[a]) / d[a], t2 = (hi - pos[a]) / d[a];
            if (t1 > t2) { double tt = t1; t1 = t2; t2 = tt; }
            if (t1 > tin) { tin = t1; ax_in = a; }
            if (t2 < tout) tout = t2;
        }
    }
    if (!(tin < tout) || tout <= 0.0 || I_h == 0) {
        memcpy(endpoint, pos, sizeof(double) * 3);
        if (T) T->escaped += I_h;
        return I_h == 0 ? END_STOP : END_MISS;
    }
    if (tin > 0.0) {
        for (int a = 0; a < 3; ++a) pos[a] += tin * d[a];
        /* the entry point lies exactly on the entry face */
        pos[ax_in] = P->org[ax_in] + (d[ax_in] > 0.0 ? 0.0 : P->n[ax_in] * P->vox[ax_in]);
    }

    /* voxel of the entry point: a point on a boundary belongs to the voxel
     * entered in the direction of travel */
    int iv[3];
    for (int a = 0; a < 3; ++a) {
        double u = (pos[a] - P->org[a]) / P->vox[a];
        double f = floor(u);
        int i = (int)f;
        if (u == f && d[a] < 0.0) i -= 1;
        if (i < 0) i = 0;
        if (i >= P->n[a]) i = P->n[a] - 1;
        iv[a] = i;
    }

    /* ---- task 2: re-trace the primary, then its secondaries --------------- */
    branch_log br = {P->sec_branch, j_first, j_end, 0, {0}, {{0}}, {{0}}, {{0}}};
    /* secondaries that start at the end of a step completed in a beam-line
     * device stay there (their energy counts as absorbed upstream) */
    while (br.j < br.end && P->sec_branch[br.j] < S.k) br.j++;
    int64_t dep_prim = 0, dep_all = 0;
    int reason = walk_trajectory(P, T, st, S.k, n_steps, k0, cum, skip, phi0, pos, iv, d, S.db, M, S.tau, S.g2, S.dep,
                                 j_first < j_end ? &br : NULL, I_h - E_sec, &dep_prim);
    memcpy(endpoint, pos, sizeof(double) * 3);
    dep_all = dep_prim;
    int bad = reason == END_STOP && dep_prim + S.up_dep != I_h - E_sec;
    if (br.n >= MAX_BRANCH) bad = 1;
    for (int q = 0; q < br.n; ++q) {
        /* a secondary leaves its branch point at (theta, phi) from the primary's direction */
        uint32_t j = br.sec[q];
        double sdb[3] = {br.db[q][0], br.db[q][1], br.db[q][2]};
        rotate(sdb, P->sec_emit[2 * j], P->sec_emit[2 * j + 1]);
        double sd[3], sp[3] = {br.pos[q][0], br.pos[q][1], br.pos[q][2]};
        for (int a = 0; a < 3; ++a) sd[a] = M[a][0] * sdb[0] + M[a][1] * sdb[1] + M[a][2] * sdb[2];
        int siv[3] = {br.iv[q][0], br.iv[q][1], br.iv[q][2]};
        const float *sst = P->sec_steps + 4 * P->sec_off[j];
        uint64_t sn = P->sec_off[j + 1] - P->sec_off[j];
        int64_t dep_s = 0;
        int sr = walk_trajectory(P, T, sst, 0, sn, UINT64_MAX, 0, 0, 0.0, sp, siv, sd, sdb, M, 0.0, 0.0, 0, NULL,
                                 sec_energy(P, j), &dep_s);
        if (sr == END_STOP && dep_s != sec_energy(P, j)) bad = 1;
        dep_all += dep_s;
    }
    if (T) T->escaped += I_h - dep_all; /* carried out of the box, absorbed upstream, or never started */
    if (bad) return -1; /* energy not conserved: oracle bug */
    return reason;
}

/* ---------------------------------------------------------------------- */
typedef struct {
    const float *steps; const uint64_t *track_off; uint32_t n_tracks;
    const float *bin_E; const uint32_t *bin_first; uint32_t n_bins;
} oracle_db_args;

static void setup(oracle_problem *P, const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                  const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                  const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                  const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                  int n_pts, double vacuum_below_hu,
                  const float *spot_pos, const float *spot_dir, const float *spot_E, const float *spot_sigma,
                  uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags)
{
    P->steps = steps; P->track_off = track_off; P->n_tracks = n_tracks;
    P->bin_E = bin_E; P->bin_first = bin_first; P->n_bins = n_bins;
    P->hu = hu;
    for (int a = 0; a < 3; ++a) { P->n[a] = dims[a]; P->vox[a] = vox[a]; P->org[a] = org[a]; }
    P->tab.hu = hu_pts; P->tab.rho = rho; P->tab.rsp = rsp; P->tab.rscp = rscp;
    P->tab.n = n_pts; P->tab.vacuum_below_hu = vacuum_below_hu;
    P->spot_pos = spot_pos; P->spot_dir = spot_dir; P->spot_E = spot_E; P->spot_sigma = spot_sigma;
    P->plan = plan; P->seed = seed; P->R = R; P->flags = flags;
    P->trace = NULL;
    P->ps_first = P->ps_count = NULL;
    P->ps_pos = P->ps_dir = P->ps_E = NULL;
    P->spot_dev = NULL;
    P->dev_par = NULL;
    P->dev_pix = NULL;
    P->dev_pix_off = NULL;
    P->sec_first = P->sec_branch = NULL;
    P->sec_off = NULL;
    P->sec_steps = P->sec_emit = NULL;
}

/* Phase-space sources for the next oracle_replay_e2x / oracle_endpoints /
 * oracle_trace_history call on this thread (see oracle_problem); NULL arrays
 * clear them.  The arrays must stay valid until that call returns. */
static _Thread_local struct {
    const uint64_t *first, *count;
    const float *pos, *dir, *E;
} g_ps;

void oracle_set_phase_space(const uint64_t *first, const uint64_t *count, const float *pos, const float *dir,
                            const float *E)
{
    g_ps.first = first; g_ps.count = count; g_ps.pos = pos; g_ps.dir = dir; g_ps.E = E;
}

/* Beam-line devices for the next calls on this thread (see oracle_problem:
 * spot_dev per spot, 16 parameters per device, pixels and their per-device
 * offsets); NULL spot_dev clears them. */
static _Thread_local struct {
    const int32_t *spot_dev;
    const double *par;
    const float *pix;
    const uint64_t *pix_off;
} g_dev;

void oracle_set_devices(const int32_t *spot_dev, const double *par, const float *pix, const uint64_t *pix_off)
{
    g_dev.spot_dev = spot_dev; g_dev.par = par; g_dev.pix = pix; g_dev.pix_off = pix_off;
}

/* The database's secondary trajectories for the next calls on this thread
 * (see oracle_problem); NULL first clears them. */
static _Thread_local struct {
    const uint32_t *first, *branch;
    const uint64_t *off;
    const float *steps, *emit;
} g_sec;

void oracle_set_secondaries(const uint32_t *first, const uint64_t *off, const float *steps, const uint32_t *branch,
                            const float *emit)
{
    g_sec.first = first; g_sec.off = off; g_sec.steps = steps; g_sec.branch = branch; g_sec.emit = emit;
}

static void use_phase_space(oracle_problem *P)
{
    if (g_ps.count) {
        P->ps_first = g_ps.first; P->ps_count = g_ps.count;
        P->ps_pos = g_ps.pos; P->ps_dir = g_ps.dir; P->ps_E = g_ps.E;
    }
    if (g_dev.spot_dev) {
        P->spot_dev = g_dev.spot_dev; P->dev_par = g_dev.par; P->dev_pix = g_dev.pix; P->dev_pix_off = g_dev.pix_off;
    }
    if (g_sec.first) {
        P->sec_first = g_sec.first; P->sec_branch = g_sec.branch; P->sec_off = g_sec.off;
        P->sec_steps = g_sec.steps; P->sec_emit = g_sec.emit;
    }
}

/*
 * Replay histories [h_begin[i], h_begin[i] + h_count[i]) of every spot i and
 * add them to the tallies E (int64) and E2 (uint64, may be NULL), plus
 * stats[0..5] = incident, escaped, steps, visits, vacuum visits, flushes
 * (int64 / uint64 bit patterns).  Threads split the flattened history range;
 * each thread tallies privately and the integer sums are added at the end,
 * which is exact.  Returns 0, or -1 if a history failed to conserve energy.
 */
int oracle_replay_e2x(const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                      const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                      const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                      const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                      int n_pts, double vacuum_below_hu,
                      const float *spot_pos, const float *spot_dir, const float *spot_E,
                      const float *spot_sigma, uint32_t n_spots,
                      const uint64_t *h_begin, const uint64_t *h_count,
                      uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags, int n_threads,
                      int64_t *E, uint64_t *E2, int64_t *stats, uint64_t *E2x);

int oracle_replay(const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                  const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                  const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                  const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                  int n_pts, double vacuum_below_hu,
                  const float *spot_pos, const float *spot_dir, const float *spot_E,
                  const float *spot_sigma, uint32_t n_spots,
                  const uint64_t *h_begin, const uint64_t *h_count,
                  uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags, int n_threads,
                  int64_t *E, uint64_t *E2, int64_t *stats)
{
    return oracle_replay_e2x(steps, track_off, n_tracks, bin_E, bin_first, n_bins, hu, dims, vox, org, hu_pts, rho,
                             rsp, rscp, n_pts, vacuum_below_hu, spot_pos, spot_dir, spot_E, spot_sigma, n_spots,
                             h_begin, h_count, plan, seed, R, flags, n_threads, E, E2, stats, NULL);
}

/* As oracle_replay; with E2x non-NULL also the per-history squared tally
 * (each history's total deposit in a voxel, rounded to 2^-12 MeV like the
 * per-visit tally, squared once). */
int oracle_replay_e2x(const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                      const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                      const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                      const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                      int n_pts, double vacuum_below_hu,
                      const float *spot_pos, const float *spot_dir, const float *spot_E,
                      const float *spot_sigma, uint32_t n_spots,
                      const uint64_t *h_begin, const uint64_t *h_count,
                      uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags, int n_threads,
                      int64_t *E, uint64_t *E2, int64_t *stats, uint64_t *E2x)
{
    oracle_problem P;
    setup(&P, steps, track_off, n_tracks, bin_E, bin_first, n_bins, hu, dims, vox, org,
          hu_pts, rho, rsp, rscp, n_pts, vacuum_below_hu, spot_pos, spot_dir, spot_E, spot_sigma,
          plan, seed, R, flags);
    use_phase_space(&P);
    size_t nvox = (size_t)dims[0] * dims[1] * dims[2];
    uint64_t *prefix = (uint64_t *)malloc(sizeof(uint64_t) * (n_spots + 1));
    prefix[0] = 0;
    for (uint32_t i = 0; i < n_spots; ++i) prefix[i + 1] = prefix[i] + h_count[i];
    uint64_t total = prefix[n_spots];
    int err = 0;
    int nt = n_threads > 0 ? n_threads : 1;
#ifdef _OPENMP
    #pragma omp parallel num_threads(nt) reduction(|:err)
#endif
    {
        int tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        oracle_tally T;
        memset(&T, 0, sizeof T);
        T.E = (int64_t *)calloc(nvox, sizeof(int64_t));
        T.E2 = E2 ? (uint64_t *)calloc(nvox, sizeof(uint64_t)) : NULL;
        if (E2x) {
            T.E2x = (uint64_t *)calloc(nvox, sizeof(uint64_t));
            T.hsum = (int64_t *)calloc(nvox, sizeof(int64_t));
            T.cap_touched = 1u << 20;
            T.touched = (size_t *)malloc(sizeof(size_t) * T.cap_touched);
        }
        uint64_t lo = total * (uint64_t)tid / (uint64_t)nth;
        uint64_t hi = total * (uint64_t)(tid + 1) / (uint64_t)nth;
        uint32_t s = 0;
        for (uint64_t g = lo; g < hi; ++g) {
            while (prefix[s + 1] <= g) ++s;
            double ep[3];
            if (replay_history(&P, s, h_begin[s] + (g - prefix[s]), &T, ep) < 0) err |= 1;
            if (E2x) { /* this history's whole deposit per voxel, squared once */
                for (size_t i = 0; i < T.n_touched; ++i) {
                    size_t v = T.touched[i];
                    uint64_t q = (uint64_t)((T.hsum[v] + 2048) >> 12);
                    T.E2x[v] += q * q;
                    T.hsum[v] = 0;
                }
                T.n_touched = 0;
                if (T.overflow) err |= 1;
            }
        }
#ifdef _OPENMP
        #pragma omp critical
#endif
        {
            for (size_t v = 0; v < nvox; ++v) E[v] += T.E[v];
            if (E2)
                for (size_t v = 0; v < nvox; ++v) E2[v] += T.E2[v];
            if (E2x)
                for (size_t v = 0; v < nvox; ++v) E2x[v] += T.E2x[v];
            stats[0] += T.incident;
            stats[1] += T.escaped;
            stats[2] += (int64_t)T.steps;
            stats[3] += (int64_t)T.visits;
            stats[4] += (int64_t)T.vacuum_visits;
            stats[5] += (int64_t)T.flushes;
        }
        free(T.E);
        free(T.E2);
        free(T.E2x);
        free(T.hsum);
        free(T.touched);
    }
    free(prefix);
    return err ? -1 : 0;
}

/* End point (cm) and end reason (0 stop, 1 escape, 2 miss, 3 stopped upstream of
 * the phantom by a beam-line device) of histories
 * h0 .. h0+n-1 of spot s.  No tallies are touched. */
int oracle_endpoints(const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                     const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                     const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                     const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                     int n_pts, double vacuum_below_hu,
                     const float *spot_pos, const float *spot_dir, const float *spot_E,
                     const float *spot_sigma, uint32_t s, uint64_t h0, uint32_t n,
                     uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags,
                     double *xyz, int32_t *reason)
{
    oracle_problem P;
    setup(&P, steps, track_off, n_tracks, bin_E, bin_first, n_bins, hu, dims, vox, org,
          hu_pts, rho, rsp, rscp, n_pts, vacuum_below_hu, spot_pos, spot_dir, spot_E, spot_sigma,
          plan, seed, R, flags);
    use_phase_space(&P);
    for (uint32_t i = 0; i < n; ++i)
        reason[i] = replay_history(&P, s, h0 + i, NULL, xyz + 3 * i);
    return 0;
}

/* The walk of one history (spot s, index h) as a list of events (test aid):
 * ev[4*i..] = (kind: 0 voxel visit, 1 vacuum voxel, 2 step end, 3 escape;
 * voxel index (step index for a step end); deposited piece in fixed point
 * (escaped remainder for an escape); exit axis of the visit or -1 if the step
 * ended inside the voxel), evd[2*i..] = (WEL consumed in the voxel, or the
 * step's accumulated sum(w*G) at a step end; geometric length moved, or the
 * deflection angle at a step end).  Returns the number of events (which may
 * exceed cap: only the first cap are written); *reason gets the end reason. */
int oracle_trace_history(const float *steps, const uint64_t *track_off, uint32_t n_tracks,
                         const float *bin_E, const uint32_t *bin_first, uint32_t n_bins,
                         const int16_t *hu, const int dims[3], const double vox[3], const double org[3],
                         const double *hu_pts, const double *rho, const double *rsp, const double *rscp,
                         int n_pts, double vacuum_below_hu,
                         const float *spot_pos, const float *spot_dir, const float *spot_E,
                         const float *spot_sigma, uint32_t s, uint64_t h,
                         uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags,
                         int64_t *ev, double *evd, int cap, int32_t *reason, double endpoint[3])
{
    oracle_problem P;
    setup(&P, steps, track_off, n_tracks, bin_E, bin_first, n_bins, hu, dims, vox, org,
          hu_pts, rho, rsp, rscp, n_pts, vacuum_below_hu, spot_pos, spot_dir, spot_E, spot_sigma,
          plan, seed, R, flags);
    use_phase_space(&P);
    oracle_trace tr = {ev, evd, cap, 0};
    P.trace = &tr;
    *reason = replay_history(&P, s, h, NULL, endpoint);
    return tr.n;
}
