/*
 * fdc.h - C ABI of the MI355X track-repeating proton dose engine (libfdc.so).
 *
 * The method (Yepes, Mirkovic, Taddei, "A GPU implementation of a
 * track-repeating algorithm for proton radiotherapy dose calculations"):
 * proton tracks pre-computed in water are re-traced through a voxelised CT
 * phantom, each step's length and scattering angle scaled by the local
 * material, and the deposited energy tallied on a voxel grid (Sections 2.2,
 * 2.3); the tally becomes dose by dividing by voxel mass, and a second tally of
 * squared deposits gives the history-by-history uncertainty of Eq. (2)
 * (Sections 2.3, 2.4).
 *
 * Conventions shared by every call
 *   - Every call returns an int status (FDC_OK or a negative FDC_E_* code); no
 *     call aborts or throws.  fdc_last_error() holds the message of the last
 *     failure on that context.
 *   - All arguments are validated before any HIP call.  Loaders are
 *     all-or-nothing: on error the previous state is unchanged.
 *   - Host arrays passed in are borrowed for the duration of the call only.
 *     Device memory belongs to the context (allocated through the allocator
 *     hook, else hipMalloc) unless a call says the caller owns it.
 *   - hip_stream is the caller's hipStream_t (NULL = the null stream).  Work is
 *     enqueued on it; fdc_run_histories and fdc_compute_dose return without
 *     waiting; calls that fill host memory synchronise the stream first.
 *   - Units: cm, MeV, rad, Gy.  Energies in the tallies are integers in units
 *     of 2^-24 MeV (fixed point), so tallies are independent of the order in
 *     which histories finish.
 *   - Arrays are x-fastest: element (ix, iy, iz) is at (iz*ny + iy)*nx + ix.
 *   - A context is used by one host thread at a time.
 */
#ifndef FDC_H
#define FDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdc_ctx fdc_ctx;
typedef struct fdc_graph fdc_graph;
typedef struct fdc_unet fdc_unet;

enum {
    FDC_OK = 0,
    FDC_E_ARG = -1,      /* null pointer, bad size, NaN, unsorted table ...          */
    FDC_E_STATE = -2,    /* call out of order (e.g. run before a database is loaded) */
    FDC_E_NOMEM = -3,    /* device or host allocation failed; state unchanged        */
    FDC_E_HIP = -4,      /* a HIP runtime call failed (message has the HIP error)    */
    FDC_E_RANGE = -5,    /* spot energy outside the database's bin energies          */
    FDC_E_FORMAT = -6,   /* malformed track database                                 */
    FDC_E_OVERFLOW = -7  /* requested histories could overflow the int64 tally       */
};

/* fdc_create's hip_device value for a context without a GPU: every argument
 * check and all host-side bookkeeping run, nothing is sent to a device, and
 * calls that must produce device results return FDC_E_STATE. */
#define FDC_NO_DEVICE (-1)

/* fdc_graph_create options */
enum {
    FDC_GRAPH_RESET_TALLIES = 1u,   /* clear the plans' tallies at the start of each launch  */
    FDC_GRAPH_DOSE = 2u             /* end each launch with dose (and variance) per plan       */
};

/* run flags */
enum {
    FDC_RUN_VARIANCE = 1u,      /* also tally squared per-visit deposits (Section 2.3)  */
    FDC_RUN_ROTATE_TRACKS = 2u, /* rotate each re-traced track by a random azimuth      */
    FDC_RUN_COUNT_WORK = 4u     /* debug: count the run's work into the plan's counters */
};

/* One stored water step (Section 2.2: direction change, length and energy loss
 * of each step): water-equivalent length, energy loss, polar and azimuthal
 * deflection applied at the end of the step.  16 bytes. */
typedef struct { float dx_cm, dE_MeV, theta_rad, phi_rad; } fdc_step;

/* A beam spot: histories start at pos + |sigma|*(n1*e1 + n2*e2) moving along
 * dir (unit), where (e1, e2) are the lateral axes of dir: e2 = normalize(dir x a),
 * e1 = e2 x dir, with a = +x if |dir.z| >= 0.9 else +z.  sigma >= 0: a pencil
 * beam, (n1, n2) standard normal; sigma < 0: a field of circular cross-section
 * (Section 2.5), (n1, n2) uniform over the unit disk, so the start points fill
 * a disk of radius -sigma uniformly.  The source region outside the phantom is
 * vacuum. */
typedef struct {
    float pos_cm[3];
    float dir[3];
    float energy_MeV;
    float sigma_cm;
    uint64_t n_histories; /* histories per fdc_run_histories call */
} fdc_spot;

/* One incident proton of a phase space (Section 2.3: the incident protons'
 * positions, directions and energies may be read from a file): start point,
 * direction (any length > 0) and kinetic energy.  32 bytes. */
typedef struct {
    float pos_cm[3];
    float dir[3];
    float energy_MeV;
    float reserved;       /* 0 */
} fdc_particle;

/* A beam-line device upstream of the phantom: an aperture and a range
 * compensator on one pixel grid (Section 4: the CPU code described them with
 * a general geometry package, the GPU code handled voxels only).  Its
 * upstream face is the plane through origin_cm perpendicular to dir (along
 * the beam, any length > 0); the grid of n[0] x n[1] pixels of pitch_cm is
 * centred on origin_cm along the lateral axes (e1, e2) of dir, defined as for
 * a spot.  A history crosses the face where its ray from the start point
 * meets it; through a closed pixel, off the grid, or if the face is not ahead
 * of it, the history stops there.  Through an open pixel with compensator
 * thickness T > 0 its track is replayed through a slab of the compensator's
 * material until its displacement along dir reaches T - water-equivalent
 * length consumed at geometric length WEL / rsp, deflections scaled by
 * sqrt(rscp / rsp), as in a voxel - and goes on towards the phantom from the
 * slab's exit face, in the middle of a stored step if it leaves there.
 * Energy deposited in the compensator, and all energy of a history stopped by
 * the device, is not deposited in the phantom: it counts as escaped. */
typedef struct {
    float origin_cm[3];
    float dir[3];
    float pitch_cm[2];
    uint32_t n[2];
    float rsp, rscp;      /* compensator material, > 0 (used where a pixel has T > 0) */
} fdc_beam_device;

typedef struct {
    uint64_t n_histories;  /* histories run on the plan since its last reset          */
    int64_t incident_fp;   /* sum of incident energies, 2^-24 MeV                      */
    int64_t deposited_fp;  /* sum of the energy tally                                  */
    int64_t escaped_fp;    /* energy not deposited in the phantom: carried out of the
                              box, or stopped or absorbed upstream by a beam-line
                              device; deposited+escaped equals incident exactly      */
} fdc_summary;

/* launch knobs; none of them changes any result bit */
typedef struct {
    uint32_t waves_per_block;   /* 1..16, default 4                                    */
    uint32_t blocks_per_cu;     /* persistent grid size = blocks_per_cu * CUs; 0 = one
                                   block per work unit (non-persistent)                */
    uint32_t tally_slots;       /* 0: flush visits with global atomics; else the size of
                                   a per-workgroup LDS sub-tally (persistent rounds;
                                   blocks_per_cu 0 is taken as 1): with tally_mode 0 a
                                   power of two 256..8192, with tally_mode 1 or 2 a
                                   multiple of 64 from 256 up to what fits              */
    uint32_t units_per_wave;    /* with tally_slots: 64-history units per wave per
                                   round (mode 2: the workgroup takes chunks of
                                   waves_per_block * units_per_wave consecutive units),
                                   1..64 (0 is taken as 1)                             */
    uint32_t tally_mode;        /* with tally_slots: 0 = hash table (voxel key, E, E2;
                                   12 or 20 B per slot) whose visits fall back to global
                                   atomics once 8 probes find no room; 1 = write-back
                                   cache of one 64-bit word (voxel | partial sum) per
                                   slot and tally (8 or 16 B per slot), a conflicting
                                   voxel evicting the old sum with one global atomic,
                                   flushed after every round; 2 = the same cache kept
                                   for the whole launch when it covers one plan (waves
                                   take units of their workgroup's chunk without
                                   barriers, one flush at the end; launches of several
                                   plans run as mode 1)                                */
    uint32_t source_order;      /* 0 = a wave unit takes 64 consecutive histories of a
                                   spot, which share one database track; 1 = the
                                   histories of each spot are processed in an order
                                   sorted by start position (chunks of 16384 of a
                                   spot's histories, each binned on up to 64 x 64
                                   cells over the spot's width in Morton order), each
                                   lane on its own track: lanes of a wave start close
                                   together, which lets the LDS cache merge deposits
                                   of broad fields.  Costs one ordering kernel per run
                                   (a lane table of 4 B per history); captured graphs
                                   capture it too.                                   */
    uint32_t reserved[2];
} fdc_launch_config;

typedef void *(*fdc_alloc_fn)(size_t bytes, void *user);
typedef void (*fdc_free_fn)(void *ptr, void *user);

/* Create a context on HIP device hip_device.  seed keys every random number
 * (Philox4x32-10); reuse_R is the number of consecutive histories of a spot
 * that re-trace one database track (the paper feeds a single stored history to
 * a whole thread group, Section 4, and re-uses it for many incident protons,
 * Section 2.3); 64 matches one wavefront.  *out receives the context.
 * hip_device == FDC_NO_DEVICE creates a validation-only context.
 * Errors: FDC_E_ARG (out NULL, reuse_R == 0), FDC_E_HIP (no such device),
 * FDC_E_NOMEM. */
int fdc_create(fdc_ctx **out, int hip_device, uint64_t seed, uint32_t reuse_R);

/* Free all device memory owned by the context and the context itself. */
int fdc_destroy(fdc_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char *fdc_last_error(const fdc_ctx *ctx);

/* Route the context's device allocations through alloc/free (e.g. a framework's
 * caching allocator).  Must be called before any loader.  Errors: FDC_E_STATE
 * if device memory was already allocated, FDC_E_ARG if only one hook is given. */
int fdc_set_allocator(fdc_ctx *ctx, fdc_alloc_fn alloc, fdc_free_fn free_fn, void *user);

/* Material table (Section 2.5: each voxel gets a material and mass density from
 * its CT number; Section 2.3: the material table holds the step-length and
 * scattering-angle scaling parameters).  Piecewise linear in HU over n_pts
 * increasing points hu_pts[]: mass density rho (g/cm^3), relative stopping power
 * rsp and relative scattering power rscp; clamped beyond the ends.  HU are
 * clamped to [-1024, 3071]; HU < vacuum_below_hu is vacuum (free flight, no
 * deposit).  Optional: the default table is used otherwise.  Applies to plans
 * loaded afterwards and to the dose of every plan.
 * Errors: FDC_E_ARG (NULL, n_pts < 2 or > 64, not increasing, negative or NaN
 * values). */
int fdc_set_hu_table(fdc_ctx *ctx, const float *hu_pts, const float *rho, const float *rsp,
                     const float *rscp, int n_pts, float vacuum_below_hu);

/* Load the water track database into device memory (Section 2.2: particle
 * trajectories stored as steps; Section 2.3: kept in GPU global memory).
 * steps[n_steps] hold the tracks back to back; track t is
 * steps[track_off[t] .. track_off[t+1]); tracks of energy bin b are
 * bin_first[b] .. bin_first[b+1]-1, bin energies bin_E_MeV[b] strictly
 * increasing.  Replaces a previously loaded database.
 * A step's energy loss must be below 128 MeV (its 2^-24 MeV fixed-point value
 * then fits 32 bits; stored steps are a few MeV).
 * Errors: FDC_E_ARG (NULL, zero counts), FDC_E_FORMAT (offsets not monotone or
 * not ending at n_steps, empty track or bin, bins not increasing, dx <= 0, dE <
 * 0, dE >= 128 MeV or any non-finite value), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_load_track_db(fdc_ctx *ctx, const fdc_step *steps, uint64_t n_steps,
                      const uint64_t *track_off, uint32_t n_tracks, const float *bin_E_MeV,
                      const uint32_t *bin_first, uint32_t n_bins, void *hip_stream);

/* Secondary trajectories of the loaded track database (Section 2.2: a stored
 * history is the set of its particles' trajectories, each broken into steps).
 * Secondary j of track t (sec_first[t] <= j < sec_first[t+1], at most 4 per
 * track) starts at the end of the track's primary step branch[j] (counted from
 * the track's first step, in order within a track), leaves at polar angle
 * emit[2j] in [0, pi] and azimuth emit[2j+1] (radians) from the primary's
 * direction there, and replays steps[sec_off[j] .. sec_off[j+1]) like a
 * primary's steps (whole, deflected at their ends, no secondaries of their
 * own).  A history replays its primary, then its secondaries from the points
 * the primary reached; their energy is part of the track's (incident energy),
 * after their branch step's in the track's order: a spot's energy skip that
 * ends inside a secondary's energy drops it and starts the primary at the next
 * step whole.  A secondary whose branch step ends inside a beam-line device is
 * absorbed there.  End-point replays (fdc_debug_endpoints) follow the primary.
 * sec_first has n_tracks + 1 entries (the database's), sec_off n_sec + 1; the
 * arrays are host memory, copied before the call returns.  Replaces previously
 * loaded secondaries; loading a track database removes them.
 * Errors: FDC_E_STATE (no track database), FDC_E_ARG (NULL arrays),
 * FDC_E_FORMAT (offsets not monotone or not ending at the counts, an empty
 * secondary, more than 4 on a track, a branch past its track's last step or
 * out of order, an angle out of range, and the step checks of
 * fdc_load_track_db), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_load_secondaries(fdc_ctx *ctx, const uint32_t *sec_first, const uint64_t *sec_off, uint32_t n_sec,
                         const fdc_step *steps, uint64_t n_sec_steps, const uint32_t *branch,
                         const float *emit, void *hip_stream);

/* The same load from a track-database file (Section 2.2: the stored water
 * histories).  Layout, all little-endian: a 104-byte header {char magic[8] =
 * "FDCTRKDB"; uint32 version = 1 or 2; uint32 n_bins, n_tracks, reserved; uint64
 * n_steps; uint64 db_seed; double physics[8] (the generator's constants, not
 * read)}, then bin_E (float x n_bins), bin_first (uint32 x n_bins+1),
 * track_off (uint64 x n_tracks+1) and the steps (fdc_step x n_steps), packed.
 * Version 2 adds secondary trajectories (fdc_load_secondaries): the header's
 * reserved word is n_sec, and after the primary steps come n_sec_steps
 * (uint64), sec_first (uint32 x n_tracks+1), sec_off (uint64 x n_sec+1),
 * branch (uint32 x n_sec), emit (float x 2 n_sec) and the secondaries' steps
 * (fdc_step x n_sec_steps), packed.
 * The file is read on the host and closed before the call returns.  Errors:
 * FDC_E_ARG (NULL path, file cannot be opened), FDC_E_FORMAT (bad magic or
 * version, a size that does not match the header, a short read, and every
 * check of fdc_load_track_db), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_load_track_db_file(fdc_ctx *ctx, const char *path, void *hip_stream);

/* Add a plan: a phantom of nx*ny*nz voxels of size voxel_cm (x, y, z) whose
 * voxel (0,0,0) starts at origin_cm, with CT numbers hu[] (host, x-fastest;
 * Section 2.3: the per-voxel material grid).  Allocates its energy and
 * squared-energy tallies (Section 2.3: the tally grid), zeroed.
 * *plan_out receives the plan id.  Errors: FDC_E_ARG (NULL, non-positive or
 * non-finite sizes, more than 2^31 voxels), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_load_phantom(fdc_ctx *ctx, int32_t *plan_out, const int16_t *hu, int nx, int ny, int nz,
                     const float voxel_cm[3], const float origin_cm[3], void *hip_stream);

/* Append n spots to a plan (Section 2.5: the incident field; Section 2.3: the
 * phase space of incident protons).  Each spot re-traces tracks of the smallest
 * bin energy >= its energy, starting inside the track where the remaining
 * energy equals the spot energy (Section 2.3, task 1).  Errors: FDC_E_ARG (bad
 * plan, NULL, non-finite values, zero direction), FDC_E_RANGE
 * (energy below the first or above the last bin energy), FDC_E_STATE (no
 * database loaded). */
int fdc_add_beam_spots(fdc_ctx *ctx, int32_t plan, const fdc_spot *spots, uint32_t n);

/* Add a beam-line device (see fdc_beam_device) to the context: pixels[n[0] *
 * n[1]] (host, e1 fastest) hold < 0 for a closed pixel, else the compensator
 * thickness in cm (0: open, no material).  Copied to the device before the
 * call returns.  *device_out receives its id (0, 1, ...).  Errors: FDC_E_ARG
 * (NULL, non-finite values, zero dir, pitch or grid size <= 0, more than 2^26
 * pixels, rsp or rscp <= 0 where a pixel has material), FDC_E_NOMEM,
 * FDC_E_HIP. */
int fdc_add_beam_device(fdc_ctx *ctx, const fdc_beam_device *device, const float *pixels, int32_t *device_out,
                        void *hip_stream);

/* Spots first_spot .. first_spot+n_spots-1 of a plan pass device `device`
 * (-1: none, the default) on their way to the phantom.  Applies to later
 * runs.  Errors: FDC_E_ARG (bad plan, spot range or device id, or a source of
 * listed protons in the range). */
int fdc_set_spot_device(fdc_ctx *ctx, int32_t plan, uint32_t first_spot, uint32_t n_spots, int32_t device);

/* Append a phase space of n protons to a plan (Section 2.3: incident protons
 * read from a file).  The protons are grouped by energy bin (the smallest bin
 * energy >= the proton's energy), bins in increasing order, list order kept
 * within a bin; each non-empty group becomes one source of the plan, numbered
 * after the plan's sources so far (spots and earlier groups), whose histories
 * per fdc_run_histories call are its protons, one pass: history h of a group
 * of m protons is its proton h mod m, so later runs re-use the protons on new
 * tracks.  Each proton starts at its own position (no lateral spread) along
 * its own direction (the beam frame of its deflections is that direction's
 * frame, as for a spot) and skips from its bin energy down to its own energy
 * on the chosen track (Section 2.3, task 1); 64 consecutive histories of a
 * group share one track.  The protons are copied to the device before the call
 * returns.  Returns the number of sources added in *n_sources_out (may be
 * NULL).  Errors: FDC_E_ARG (bad plan, NULL with n > 0, non-finite values,
 * zero direction, reserved != 0), FDC_E_RANGE (an energy outside the bin
 * energies), FDC_E_STATE (no database loaded), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_add_phase_space(fdc_ctx *ctx, int32_t plan, const fdc_particle *particles, uint64_t n,
                        uint32_t *n_sources_out, void *hip_stream);

/* The same from a phase-space file: a 32-byte little-endian header {char
 * magic[8] = "FDCPHSP1"; uint32 version = 1; uint32 record_bytes = 32; uint64
 * n; uint64 reserved = 0} followed by n fdc_particle records.  The file is
 * read on the host and closed before the call returns.  Errors: as
 * fdc_add_phase_space, plus FDC_E_ARG (NULL path, file cannot be opened) and
 * FDC_E_FORMAT (bad magic, version or record size, a size that does not match
 * the header, a short read). */
int fdc_add_phase_space_file(fdc_ctx *ctx, int32_t plan, const char *path, uint32_t *n_sources_out,
                             void *hip_stream);

/* One pass of the method over n_plans plans in a single launch (Section 2.3:
 * every incident proton is an independent thread re-tracing a stored
 * history): every spot of every listed plan runs its n_histories more
 * histories.  A history is identified by (plan, spot, h) where h continues
 * across calls; that identity keys every random number, so tallies do not
 * depend on launch configuration, batching or call splitting.  flags:
 * FDC_RUN_*.  Asynchronous on hip_stream.  Errors: FDC_E_ARG (bad or repeated
 * plan id), FDC_E_STATE (no database), FDC_E_OVERFLOW (the plan's histories
 * times the largest bin energy could exceed the int64 tally), FDC_E_NOMEM,
 * FDC_E_HIP. */
int fdc_run_histories(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags,
                      void *hip_stream);

/* fdc_run_histories for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * pass with the same kernels and bit-identical tallies, but its work table,
 * persistent-queue counter and start-position lane table live in a scratch
 * array of 32 MiB that the library holds statically on every device it runs
 * on (until the process ends), and the work table is built on the device from
 * the spot table, so the call allocates nothing, on the device or the host.
 * Limits: at most 64 plans, 16384 spots with histories, and with
 * source_order 1 at most 120,709 wave units (about 7.7e6 histories) per call.
 * The plan and spot tables must be current: after loading phantoms or adding
 * spots, call fdc_prepare_run (or any fdc_run_histories) first.  All calls of
 * this function on one device share the scratch: calls that overlap in time
 * on one GPU (different streams, or different contexts on one device) race;
 * calls on one stream are ordered.  Asynchronous on hip_stream.  Errors: as
 * fdc_run_histories, plus FDC_E_RANGE (beyond the limits above) and
 * FDC_E_STATE (tables not current, no device). */
int fdc_run_histories_noalloc(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags,
                              void *hip_stream);

/* Bring the device plan and spot tables up to date (may allocate; a no-op
 * when nothing changed).  fdc_run_histories does this by itself.  Errors:
 * FDC_E_ARG, FDC_E_NOMEM, FDC_E_HIP, FDC_E_RANGE / FDC_E_STATE (a spot no
 * longer valid for the loaded database). */
int fdc_prepare_run(fdc_ctx *ctx);

/* Capture one fdc_run_histories pass over n_plans plans (plus, with options,
 * clearing the tallies first and computing dose and variance after) as a HIP
 * graph, for repeated launches with one call each.  The plans' spots, the
 * launch configuration and the outputs are fixed at capture; every launch runs
 * each spot's n_histories NEXT histories (the history counters live on the
 * device and advance inside the graph), so replays are new work with the same
 * random-number identity as eager runs.  dose_dev / var_dev: arrays of
 * n_plans DEVICE pointers (nx*ny*nz doubles each, either array may be NULL)
 * used with FDC_GRAPH_DOSE.  No memory is allocated by a launch.  A graph
 * becomes stale when a phantom, spots or a database is loaded afterwards
 * (launch then returns FDC_E_STATE).  Errors: as fdc_run_histories, plus
 * FDC_E_ARG (bad options), FDC_E_STATE (no device; variance output without
 * FDC_RUN_VARIANCE history), FDC_E_HIP. */
int fdc_graph_create(fdc_ctx *ctx, const int32_t *plans, uint32_t n_plans, uint32_t flags, uint32_t options,
                     double *const *dose_dev, double *const *var_dev, fdc_graph **out);

/* Launch a captured graph on hip_stream (asynchronous).  Errors: FDC_E_ARG,
 * FDC_E_STATE (stale graph), FDC_E_OVERFLOW (without FDC_GRAPH_RESET_TALLIES,
 * as fdc_run_histories), FDC_E_HIP. */
int fdc_graph_launch(fdc_graph *graph, void *hip_stream);

/* Wait for the device, then free the graph and its work table. */
int fdc_graph_destroy(fdc_graph *graph);

/* Checkpoint and resume of a plan: its tallies (E, E2), summary (incident,
 * escaped, histories run) and each source's next-history counter, as one
 * host buffer of fdc_plan_state_bytes bytes (a 48-byte header {char
 * magic[8] = "FDCSTATE"; uint32 version = 1, var_complete; uint64 nvox,
 * n_sources, n_hist, reserved}, the summary words (8 x uint64), the counters
 * (uint64 per source) and E, E2 (uint64 per voxel), little-endian).  Random
 * numbers are keyed by counters and the tallies are integers, so a plan
 * restored into a context with the same database, seed, phantom and sources
 * continues exactly as the saved run would have: run(N), save, restore
 * elsewhere, run(N) equals run(2N) bit for bit.  Save and restore are
 * synchronous on hip_stream (order them after the runs they cover on the same
 * stream); the caller owns buf.  A context without a device saves zero
 * tallies and restores the counters only.  Errors: FDC_E_ARG (NULL, no such
 * plan, a save buffer of the wrong size), FDC_E_FORMAT (restore: bad magic or
 * version, a voxel or source count other than the plan's, a size that does
 * not match), FDC_E_HIP. */
int fdc_plan_state_bytes(fdc_ctx *ctx, int32_t plan, uint64_t *bytes);
int fdc_save_plan_state(fdc_ctx *ctx, int32_t plan, void *buf, uint64_t bytes, void *hip_stream);
int fdc_restore_plan_state(fdc_ctx *ctx, int32_t plan, const void *buf, uint64_t bytes, void *hip_stream);

/* The work counters of a plan (a debug aid for the roofline's per-history byte
 * counts): counts[0] = steps started in the phantom, counts[1] = non-vacuum
 * voxel pieces (Section 2.3 task 2: a step consumed voxel by voxel), counts[2]
 * = deposits flushed to the tallies, summed over the plan's runs with
 * FDC_RUN_COUNT_WORK since it was loaded or last reset.  Such a run takes the
 * global-atomic kernel (one wave per 64-history unit) whatever the launch
 * configuration, with tallies bitwise equal to any other run's.  Vacuum
 * voxels crossed in free flight are not pieces.  Synchronous on hip_stream;
 * a context without a device reports zeros.  Errors: FDC_E_ARG (NULL, no
 * such plan), FDC_E_HIP. */
int fdc_read_work_counts(fdc_ctx *ctx, int32_t plan, uint64_t counts[3], void *hip_stream);

/* Zero a plan's tallies, summary and work counters (asynchronous).  The history counters keep
 * running unless rewind is non-zero, in which case the next run repeats the
 * same histories from h = 0.  Errors: FDC_E_ARG. */
int fdc_reset_plan(fdc_ctx *ctx, int32_t plan, int rewind, void *hip_stream);

/* Dose per primary and its Eq. (2) variance into caller-owned DEVICE arrays of
 * nx*ny*nz doubles (either may be NULL), asynchronously.  Dose = deposited
 * energy / voxel mass / N (Section 2.3), N the plan's histories; variance =
 * (S2/N - (S1/N)^2)/(N-1) with S1, S2 the sums of per-history dose and squared
 * dose (Eq. (2), summed over all N histories).  Vacuum voxels get 0.
 * Errors: FDC_E_ARG, FDC_E_STATE (variance asked but a run without
 * FDC_RUN_VARIANCE touched the plan, or no history run), FDC_E_HIP. */
int fdc_compute_dose(fdc_ctx *ctx, int32_t plan, double *dose_dev, double *var_dev,
                     void *hip_stream);

/* As fdc_compute_dose, into HOST arrays, plus the raw tallies (raw_E int64,
 * raw_E2 uint64, nx*ny*nz each) and the summary; any pointer may be NULL.
 * Synchronises hip_stream.  Errors as fdc_compute_dose. */
int fdc_read_dose_and_variance(fdc_ctx *ctx, int32_t plan, double *dose_gy_per_primary,
                               double *var_gy2, int64_t *raw_E, uint64_t *raw_E2,
                               fdc_summary *sum, void *hip_stream);

/* Replay histories h0 .. h0+n-1 of spot `spot` of a plan without tallying and
 * return their end points (host xyz_out[3n], cm) and end reasons (host
 * reason_out[n]: 0 stopped, 1 escaped the phantom, 2 missed it, 3 stopped
 * upstream of it by a beam-line device).  Uses the
 * same kernel code as fdc_run_histories.  Synchronises hip_stream.
 * Errors: FDC_E_ARG, FDC_E_STATE, FDC_E_HIP. */
int fdc_debug_endpoints(fdc_ctx *ctx, int32_t plan, uint32_t spot, uint64_t h0, uint32_t n,
                        uint32_t flags, float *xyz_out, int32_t *reason_out, void *hip_stream);

/* Device Philox4x32-10 (Salmon et al., SC'11) of n counters ctr[4n] under the
 * context seed, into out[4n] (host arrays).  For testing the generator.
 * Synchronises hip_stream.  Errors: FDC_E_ARG, FDC_E_HIP. */
int fdc_debug_philox(fdc_ctx *ctx, const uint32_t *ctr, uint32_t *out, uint32_t n, void *hip_stream);

/* The material table as staged on the device: for HU index i = HU + 1024,
 * i in 0..4095, rsp_out[i], g_out[i] = rscp/rsp and rho_out[i] (host arrays of
 * 4096 floats; vacuum entries have rsp = g = 0).  Synchronises hip_stream. */
int fdc_debug_material(fdc_ctx *ctx, float *rsp_out, float *g_out, float *rho_out, void *hip_stream);

/* Launch knobs for fdc_run_histories (see fdc_launch_config).  Results are
 * bitwise identical for every valid setting.  Errors: FDC_E_ARG (out of range,
 * or an LDS sub-tally that does not fit next to the 32 KB material table in
 * 160 KB; with the squared-energy tally the size is checked again at run
 * time). */
int fdc_set_launch_config(fdc_ctx *ctx, const fdc_launch_config *cfg);

/* Mean dose uncertainty (Section 2.4): the mean of sqrt(var)/dose over the
 * plan's non-vacuum voxels whose dose exceeds frac * Dmax (frac = 0.5 in the
 * paper), Dmax taken over non-vacuum voxels.  dose_dev / var_dev: DEVICE
 * arrays of the plan's voxel count (e.g. from fdc_compute_dose).  Host
 * outputs: *mean_out, and optionally the number of voxels averaged and Dmax.
 * Reductions run in a fixed order (reproducible).  Synchronises hip_stream.
 * Errors: FDC_E_ARG, FDC_E_STATE (no device), FDC_E_NOMEM, FDC_E_HIP. */
int fdc_mean_uncertainty(fdc_ctx *ctx, int32_t plan, const double *dose_dev, const double *var_dev, double frac,
                         double *mean_out, uint64_t *n_out, double *dmax_out, void *hip_stream);

/* Batch uncertainty, Eq. (1): for n_batches >= 2 dose arrays stored back to
 * back in doses_dev (DEVICE, n_batches * n_vox doubles), per voxel the mean
 * and sqrt(sum_i (D_i - mean)^2 / (n (n - 1))) into DEVICE arrays mean_dev /
 * sigma_dev (either may be NULL).  Asynchronous.  Errors: FDC_E_ARG,
 * FDC_E_STATE (no device), FDC_E_HIP. */
int fdc_batch_uncertainty(fdc_ctx *ctx, const double *doses_dev, uint32_t n_batches, uint64_t n_vox,
                          double *mean_dev, double *sigma_dev, void *hip_stream);

/* Gamma index (Low et al. 1998; Section 2.4 uses 3%/3 mm, pass when gamma <=
 * 1) of the evaluated dose eval_dev against the reference ref_dev (DEVICE
 * arrays on the plan's grid).  Global dose criterion dose_frac * Dmax(ref),
 * distance criterion dta_cm; reference voxels that are vacuum or below
 * cutoff_frac * Dmax are not evaluated.  For each evaluated voxel, gamma is the
 * minimum over points of the evaluated dose upsampled twice per axis by
 * trilinear interpolation within search_cm of
 * sqrt(r^2 / dta^2 + (D_e - D_r)^2 / (dose_frac * Dmax)^2).  gamma_dev
 * (DEVICE floats, may be NULL) receives gamma per voxel (-1 where not
 * evaluated); *pass_rate_out the fraction of evaluated voxels with gamma <= 1.
 * Synchronises hip_stream.  Errors: FDC_E_ARG, FDC_E_STATE, FDC_E_NOMEM,
 * FDC_E_HIP. */
int fdc_gamma_index(fdc_ctx *ctx, int32_t plan, const double *ref_dev, const double *eval_dev, double dose_frac,
                    double dta_cm, double cutoff_frac, double search_cm, float *gamma_dev, double *pass_rate_out,
                    uint64_t *n_eval_out, void *hip_stream);

/* Mass density (g/cm^3) of every voxel of a plan from its HU (Section 2.5)
 * into a DEVICE float array of nx*ny*nz.  Asynchronous.  Errors: FDC_E_ARG,
 * FDC_E_STATE (no device), FDC_E_HIP. */
int fdc_density(fdc_ctx *ctx, int32_t plan, float *rho_dev, void *hip_stream);

/* Denoiser input of a plan (DEVICE arrays): out[0][v] = dose[v] * scale
 * (scale = 1/Dmax of that dose), out[1][v] = rho[v] / 2.  Asynchronous. */
int fdc_denoise_input(fdc_ctx *ctx, int32_t plan, const double *dose_dev, const float *rho_dev, double scale,
                      float *out_dev, void *hip_stream);

/* Number of compute units of the context's device (for launch sizing). */
int fdc_device_cus(fdc_ctx *ctx, int *cus);

/* Measurement aid: with timing on, every fdc_run_histories records a pair of
 * HIP events on its stream around the transport kernel alone (not the source
 * ordering, the queue reset or the history-counter update); the context keeps
 * the last 64 pairs.  fdc_set_timing(ctx, 1) turns it on and forgets earlier
 * pairs (0 turns it off).  fdc_transport_times writes the kernel durations
 * (milliseconds) of the last n timed runs, oldest first, into the host array
 * ms[n]; it waits for the last one to finish.  Captured graphs are not timed.
 * Errors: FDC_E_ARG (NULL), FDC_E_STATE (no device; n above the runs timed
 * and kept), FDC_E_HIP. */
int fdc_set_timing(fdc_ctx *ctx, int on);
int fdc_transport_times(fdc_ctx *ctx, float *ms, uint32_t n);

/* ---------------------------------------------------------------------------
 * Dose denoiser: a 3-level 3D U-Net mapping (low-history dose, density) to a
 * high-history dose, trained and run with BF16 MFMA kernels accumulating in
 * FP32.  Layers (channels-first notation): conv3 2->16, 16->16 | avg-pool 2 |
 * conv3 16->32, 32->32 | pool | conv3 32->64, 64->64 | transposed conv 2x2x2
 * stride 2 64->32, concat with the 32-channel encoder output | conv3 64->32,
 * 32->32 | transposed conv 32->16, concat | conv3 32->16, 16->16 | conv1 16->1,
 * plus the input dose (residual).  conv3 = 3x3x3 cross-correlation, zero
 * padding 1, ReLU after every conv3.  Loss: mean squared error.
 * Parameters: one flat FP32 vector of fdc_unet_num_params() values, per layer
 * in the order above: weights in C order of [cout][cin][3][3][3] (conv3),
 * [cin][cout][2][2][2] (transposed) or [cout][cin] (conv1), then biases.
 * ------------------------------------------------------------------------- */

/* Number of parameters of the network (339 681). */
int64_t fdc_unet_num_params(void);

/* A network instance for volumes of nx*ny*nz voxels (each a multiple of 4),
 * with its activation, gradient and Adam buffers.  Parameters start at zero:
 * set them with fdc_unet_set_params.  Errors: FDC_E_ARG, FDC_E_HIP, FDC_E_NOMEM. */
int fdc_unet_create(fdc_unet **out, int hip_device, int nx, int ny, int nz);
int fdc_unet_destroy(fdc_unet *u);
const char *fdc_unet_last_error(const fdc_unet *u);

/* Copy the flat parameter vector in (host, FP32), clear the Adam moments and
 * pack the bf16 operands.  Synchronises hip_stream.  FDC_E_ARG on NULL/NaN. */
int fdc_unet_set_params(fdc_unet *u, const float *host_params, void *hip_stream);
/* He-normal initialisation (std sqrt(2 / fan_in); the head x 0.1; biases 0)
 * from a seeded host generator, then as fdc_unet_set_params. */
int fdc_unet_init_params(fdc_unet *u, uint64_t seed, void *hip_stream);
/* Copy the parameters / the gradients of the last fdc_unet_backward out to
 * host arrays of fdc_unet_num_params() floats.  Synchronise hip_stream. */
int fdc_unet_get_params(fdc_unet *u, float *host_params, void *hip_stream);
int fdc_unet_get_grads(fdc_unet *u, float *host_grads, void *hip_stream);

/* Inference: in_dev = DEVICE FP32 [2][nz][ny][nx] (channel 0 the dose, 1 the
 * density input), out_dev = DEVICE FP32 [nz][ny][nx].  Asynchronous. */
int fdc_unet_forward(fdc_unet *u, const float *in_dev, float *out_dev, void *hip_stream);

/* Forward, mean-squared-error loss against target_dev (DEVICE FP32
 * [nz][ny][nx]) and backward: the gradient of the loss with respect to every
 * parameter is left in the instance (FP32).  out_dev (may be NULL) receives
 * the prediction; loss_host (may be NULL; then the call is asynchronous)
 * the loss, after synchronising hip_stream.  Errors: FDC_E_ARG, FDC_E_HIP. */
int fdc_unet_backward(fdc_unet *u, const float *in_dev, const float *target_dev, float *out_dev,
                      double *loss_host, void *hip_stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected) on the FP32 parameters
 * with the last gradients, then re-pack the bf16 operands.  Asynchronous. */
int fdc_unet_adam(fdc_unet *u, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Testing aid: copy internal bf16 buffer `index` (0..26: x, e1a, c1, p1, e2a,
 * c2, p2, ma, m, d2a, d2, d1a, d1, then the gradients gd1, gd1a, gc1, gd2,
 * gd2a, gc2, gm, gma, gp2, ge2, ge2a, gp1, ge1, ge1a; channels-last,
 * *pitch values per voxel) to host_out (NULL: sizes only).  Synchronises. */
int fdc_unet_debug_buffer(fdc_unet *u, int index, uint16_t *host_out, int64_t *n_voxels, int32_t *pitch,
                          void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FDC_H */
