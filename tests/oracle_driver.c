/* Stand-alone driver of the CPU oracle for sanitizer builds (AddressSanitizer
 * and UndefinedBehaviorSanitizer): reads a track-database file and a small
 * problem written by the test, replays every spot (with the literal Eq. (2)
 * tally), traces and end-points a few histories, and prints the integer
 * results so that the test can compare them with the ordinary build.
 * Usage: oracle_driver db.bin problem.bin */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_replay_e2x(const float *steps, const uint64_t *track_off, uint32_t n_tracks, const float *bin_E,
                      const uint32_t *bin_first, uint32_t n_bins, const int16_t *hu, const int dims[3],
                      const double vox[3], const double org[3], const double *hu_pts, const double *rho,
                      const double *rsp, const double *rscp, int n_pts, double vacuum_below_hu,
                      const float *spot_pos, const float *spot_dir, const float *spot_E, const float *spot_sigma,
                      uint32_t n_spots, const uint64_t *h_begin, const uint64_t *h_count, uint32_t plan,
                      uint64_t seed, uint32_t R, uint32_t flags, int n_threads, int64_t *E, uint64_t *E2,
                      int64_t *stats, uint64_t *E2x);
int oracle_endpoints(const float *steps, const uint64_t *track_off, uint32_t n_tracks, const float *bin_E,
                     const uint32_t *bin_first, uint32_t n_bins, const int16_t *hu, const int dims[3],
                     const double vox[3], const double org[3], const double *hu_pts, const double *rho,
                     const double *rsp, const double *rscp, int n_pts, double vacuum_below_hu,
                     const float *spot_pos, const float *spot_dir, const float *spot_E, const float *spot_sigma,
                     uint32_t s, uint64_t h0, uint32_t n, uint32_t plan, uint64_t seed, uint32_t R, uint32_t flags,
                     double *xyz, int32_t *reason);
int oracle_trace_history(const float *steps, const uint64_t *track_off, uint32_t n_tracks, const float *bin_E,
                         const uint32_t *bin_first, uint32_t n_bins, const int16_t *hu, const int dims[3],
                         const double vox[3], const double org[3], const double *hu_pts, const double *rho,
                         const double *rsp, const double *rscp, int n_pts, double vacuum_below_hu,
                         const float *spot_pos, const float *spot_dir, const float *spot_E,
                         const float *spot_sigma, uint32_t s, uint64_t h, uint32_t plan, uint64_t seed, uint32_t R,
                         uint32_t flags, int64_t *ev, double *evd, int cap, int32_t *reason, double endpoint[3]);

static void *read_exact(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    unsigned char hdr[104];
    if (fread(hdr, 1, sizeof hdr, f) != sizeof hdr) return 2;
    uint32_t nb, nt;
    uint64_t ns;
    memcpy(&nb, hdr + 12, 4);
    memcpy(&nt, hdr + 16, 4);
    memcpy(&ns, hdr + 24, 8);
    float *bin_E = read_exact(f, 4 * (size_t)nb);
    uint32_t *bin_first = read_exact(f, 4 * ((size_t)nb + 1));
    uint64_t *off = read_exact(f, 8 * ((size_t)nt + 1));
    float *steps = read_exact(f, 16 * (size_t)ns);
    fclose(f);

    /* problem: int32 dims[3], double vox[3], org[3], int32 n_pts, double
     * table[4][n_pts], double vacuum, uint32 n_spots, float pos[3n], dir[3n],
     * E[n], sigma[n], uint64 count[n], int16 hu[nvox] */
    f = fopen(argv[2], "rb");
    if (!f) return 2;
    int dims[3];
    double vox[3], org[3], vac;
    int32_t n_pts;
    uint32_t n_spots;
    if (fread(dims, 4, 3, f) != 3 || fread(vox, 8, 3, f) != 3 || fread(org, 8, 3, f) != 3 ||
        fread(&n_pts, 4, 1, f) != 1)
        return 2;
    double *tab = read_exact(f, 8 * 4 * (size_t)n_pts);
    if (fread(&vac, 8, 1, f) != 1 || fread(&n_spots, 4, 1, f) != 1) return 2;
    float *pos = read_exact(f, 12 * (size_t)n_spots), *dir = read_exact(f, 12 * (size_t)n_spots);
    float *E = read_exact(f, 4 * (size_t)n_spots), *sig = read_exact(f, 4 * (size_t)n_spots);
    uint64_t *cnt = read_exact(f, 8 * (size_t)n_spots);
    const size_t nvox = (size_t)dims[0] * dims[1] * dims[2];
    int16_t *hu = read_exact(f, 2 * nvox);
    fclose(f);

    uint64_t *h0 = calloc(n_spots, 8);
    int64_t *Et = calloc(nvox, 8);
    uint64_t *E2 = calloc(nvox, 8), *E2x = calloc(nvox, 8);
    int64_t stats[6] = {0};
    const double *t = tab;
    int rc = oracle_replay_e2x(steps, off, nt, bin_E, bin_first, nb, hu, dims, vox, org, t, t + n_pts, t + 2 * n_pts,
                               t + 3 * n_pts, n_pts, vac, pos, dir, E, sig, n_spots, h0, cnt, 0, 1, 64, 1, 2, Et, E2,
                               stats, E2x);
    uint64_t hE = 1469598103934665603ull, hE2 = hE, hE2x = hE;
    for (size_t v = 0; v < nvox; ++v) {
        hE = (hE ^ (uint64_t)Et[v]) * 1099511628211ull;
        hE2 = (hE2 ^ E2[v]) * 1099511628211ull;
        hE2x = (hE2x ^ E2x[v]) * 1099511628211ull;
    }
    printf("replay rc=%d incident=%lld escaped=%lld steps=%lld visits=%lld vacuum=%lld flushes=%lld\n", rc,
           (long long)stats[0], (long long)stats[1], (long long)stats[2], (long long)stats[3], (long long)stats[4],
           (long long)stats[5]);
    printf("hash E=%016llx E2=%016llx E2x=%016llx\n", (unsigned long long)hE, (unsigned long long)hE2,
           (unsigned long long)hE2x);
    double xyz[3 * 16];
    int32_t reason[16];
    oracle_endpoints(steps, off, nt, bin_E, bin_first, nb, hu, dims, vox, org, t, t + n_pts, t + 2 * n_pts,
                     t + 3 * n_pts, n_pts, vac, pos, dir, E, sig, 0, 5, 16, 0, 1, 64, 2, xyz, reason);
    for (int i = 0; i < 16; ++i) printf("end %d %.9f %.9f %.9f\n", reason[i], xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
    int64_t ev[4 * 64];
    double evd[2 * 64], ep[3];
    int32_t why;
    const int n = oracle_trace_history(steps, off, nt, bin_E, bin_first, nb, hu, dims, vox, org, t, t + n_pts,
                                       t + 2 * n_pts, t + 3 * n_pts, n_pts, vac, pos, dir, E, sig, 0, 3, 0, 1, 64, 0,
                                       ev, evd, 64, &why, ep);
    printf("trace n=%d reason=%d\n", n, why);
    free(bin_E); free(bin_first); free(off); free(steps); free(tab); free(pos); free(dir); free(E); free(sig);
    free(cnt); free(hu); free(h0); free(Et); free(E2); free(E2x);
    return rc == 0 ? 0 : 1;
}
