// The library's per-history walk (replay_history in transport.hip: source
// sample, start step, FP32 voxel walk with vacuum free flight, deflection)
// compiled for the host and run one history at a time, so that the test can
// compare its tallies and end points with the oracle's and, built with
// AddressSanitizer, check that every voxel, step-record and table access stays
// inside its array.  The device-side tables (material table, voxel words with
// vacuum-skip bits, stored steps in their load-time form, spot records) are
// built here from the raw inputs by restating what the loaders do.
//
// Usage: walk_host db.bin problem.bin out_prefix
//   problem.bin: int32 dims[3]; double vox[3], org[3]; int32 n_pts; double
//   table[4][n_pts]; double vacuum; uint32 n_spots; float pos[3n], dir[3n],
//   E[n], sigma[n]; uint64 count[n]; int16 hu[nvox]; uint32 flags; uint32 R
// Writes out_prefix.E (int64 per voxel), .E2 (uint64), .ep (per history: x, y,
// z as float, reason as int32) and prints "incident escaped".
#include "transport.hip"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace fdc;

namespace {

struct HostSink {
    std::vector<long long> *E;
    std::vector<unsigned long long> *E2;
    bool var;
    void add(uint32_t v, uint32_t, long long acc) const
    {
        (*E)[v] += acc;
        if (var) {
            const unsigned long long q = (unsigned long long)((acc + 2048) >> 12);
            (*E2)[v] += q * q;
        }
    }
};

template <class T>
std::vector<T> read_vec(FILE *f, size_t n)
{
    std::vector<T> v(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short read\n");
        std::exit(2);
    }
    return v;
}

double table_value(const std::vector<double> &t, int n, int col, double h)
{
    // rows of (hu, rho, rsp, rscp), stored column-major in the problem file
    const double *hu = t.data();
    const double *val = t.data() + (size_t)col * n;
    if (h <= hu[0]) return val[0];
    if (h >= hu[n - 1]) return val[n - 1];
    int j = 0;
    while (!(h < hu[j + 1])) ++j;
    return val[j] + (val[j + 1] - val[j]) * (h - hu[j]) / (hu[j + 1] - hu[j]);
}

} // namespace

int main(int argc, char **argv)
{
    if (argc != 4) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    unsigned char hdr[104];
    if (std::fread(hdr, 1, sizeof hdr, f) != sizeof hdr) return 2;
    uint32_t nb, nt;
    uint64_t ns;
    std::memcpy(&nb, hdr + 12, 4);
    std::memcpy(&nt, hdr + 16, 4);
    std::memcpy(&ns, hdr + 24, 8);
    auto bin_E = read_vec<float>(f, nb);
    auto bin_first = read_vec<uint32_t>(f, nb + 1);
    auto off = read_vec<unsigned long long>(f, nt + 1);
    auto raw = read_vec<float>(f, 4 * ns);
    std::fclose(f);

    f = std::fopen(argv[2], "rb");
    if (!f) return 2;
    auto dims = read_vec<int32_t>(f, 3);
    auto vox = read_vec<double>(f, 3);
    auto org = read_vec<double>(f, 3);
    const int n_pts = read_vec<int32_t>(f, 1)[0];
    auto tab = read_vec<double>(f, 4 * (size_t)n_pts);
    const double vac = read_vec<double>(f, 1)[0];
    const uint32_t n_spots = read_vec<uint32_t>(f, 1)[0];
    auto pos = read_vec<float>(f, 3 * (size_t)n_spots);
    auto dir = read_vec<float>(f, 3 * (size_t)n_spots);
    auto En = read_vec<float>(f, n_spots);
    auto sig = read_vec<float>(f, n_spots);
    auto cnt = read_vec<uint64_t>(f, n_spots);
    const size_t nvox = (size_t)dims[0] * dims[1] * dims[2];
    auto hu = read_vec<int16_t>(f, nvox);
    const uint32_t flags = read_vec<uint32_t>(f, 1)[0];
    const uint32_t R = read_vec<uint32_t>(f, 1)[0];
    std::fclose(f);

    // stored steps in their load-time form, and each track's total energy
    std::vector<float4> steps(ns);
    for (uint64_t k = 0; k < ns; ++k) {
        const float *r = &raw[4 * k];
        float sp, cp;
        sincosf(r[3], &sp, &cp);
        steps[k] = make_float4(r[0], __builtin_bit_cast(float, (int)to_fp(r[1])), r[2] * cp, r[2] * sp);
    }
    std::vector<long long> T(nt, 0);
    for (uint32_t t = 0; t < nt; ++t)
        for (unsigned long long k = off[t]; k < off[t + 1]; ++k) T[t] += to_fp(raw[4 * k + 1]);

    // material table and voxel words (HU index | vacuum skip << 12)
    std::vector<float2> lut(kLutSize);
    for (int i = 0; i < kLutSize; ++i) {
        const double h = (double)(i + kHuMin);
        const double s = table_value(tab, n_pts, 2, h), c = table_value(tab, n_pts, 3, h);
        lut[i] = (h < vac || !(s > 0.0)) ? make_float2(0.f, 0.f) : make_float2((float)s, (float)(c / s));
    }
    std::vector<uint16_t> idx(nvox);
    for (size_t v = 0; v < nvox; ++v) {
        const int h = std::min(std::max((int)hu[v], kHuMin), kHuMin + kLutSize - 1) - kHuMin;
        idx[v] = (uint16_t)(h | ((lut[h].x == 0.f ? kMaxSkip : 0u) << kHuBits));
    }
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    for (uint32_t pass = 0; pass < kMaxSkip; ++pass) {
        std::vector<uint16_t> nxt = idx;        // Jacobi passes: the same fixed point as the in-place kernel
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t v = ((size_t)z * ny + y) * nx + x;
                    uint32_t best = vacuum_skip(idx[v]);
                    if (best <= 1u) continue;
                    for (int dz = -1; dz <= 1; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const int xx = x + dx, yy = y + dy, zz = z + dz;
                                if (xx < 0 || yy < 0 || zz < 0 || xx >= nx || yy >= ny || zz >= nz) continue;
                                best = std::min(best, vacuum_skip(idx[((size_t)zz * ny + yy) * nx + xx]) + 1u);
                            }
                    nxt[v] = (uint16_t)(hu_index(idx[v]) | (best << kHuBits));
                }
        idx.swap(nxt);
    }

    DevPlan pl{};
    pl.idx = idx.data();
    for (int q = 0; q < 3; ++q) {
        pl.n[q] = dims[q];
        pl.vox[q] = (float)vox[q];
        pl.inv_vox[q] = 1.f / (float)vox[q];
        pl.org[q] = (float)org[q];
        pl.vox_d[q] = (double)(float)vox[q];
        pl.org_d[q] = (double)(float)org[q];
    }
    TransportArgs a{};
    a.steps = steps.data();
    a.track_off = off.data();
    a.track_T = T.data();
    a.bin_first = bin_first.data();
    a.seed_lo = 1;
    a.seed_hi = 0;
    a.R = R;
    a.flags = flags;

    std::vector<long long> E(nvox, 0);
    std::vector<unsigned long long> E2(nvox, 0);
    const HostSink sink{&E, &E2, (flags & kFlagVariance) != 0};
    long long incident = 0, escaped = 0;
    WorkCount work{0u, 0u, 0u};         // steps, voxel pieces and flushes of every history
    std::vector<float> ep_xyz;
    std::vector<int> ep_reason;
    for (uint32_t s = 0; s < n_spots; ++s) {
        DevSpot sp{};
        sp.dev = -1;                                   // no beam-line device
        double d[3] = {dir[3 * s], dir[3 * s + 1], dir[3 * s + 2]};
        const double l = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (double &x : d) x /= l;
        double ax[3] = {0.0, 0.0, 1.0};
        if (std::fabs(d[2]) >= 0.9) { ax[0] = 1.0; ax[2] = 0.0; }
        double e2[3] = {d[1] * ax[2] - d[2] * ax[1], d[2] * ax[0] - d[0] * ax[2], d[0] * ax[1] - d[1] * ax[0]};
        const double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        for (double &x : e2) x /= l2;
        const double e1[3] = {e2[1] * d[2] - e2[2] * d[1], e2[2] * d[0] - e2[0] * d[2], e2[0] * d[1] - e2[1] * d[0]};
        float wc[16] = {};
        for (int q = 0; q < 3; ++q) {
            sp.pos[q] = pos[3 * s + q];
            sp.e1[q] = e1[q];
            sp.e2[q] = e2[q];
            sp.d[q] = d[q];
            sp.m[3 * q + 0] = (float)e1[q];
            sp.m[3 * q + 1] = (float)e2[q];
            sp.m[3 * q + 2] = (float)d[q];
        }
        for (int q = 0; q < 9; ++q) wc[q] = sp.m[q];
        for (int q = 0; q < 3; ++q) wc[9 + q] = pl.inv_vox[q];
        sp.sigma = sig[s];
        uint32_t b = 0;
        while (b < nb && bin_E[b] < En[s]) ++b;
        sp.bin = b;
        sp.plan = 0;
        sp.spot = s;
        sp.skip = to_fp(bin_E[b]) - to_fp(En[s]);
        sp.n_hist = cnt[s];
        float xyz[3];
        int reason = 0;
        for (uint64_t h = 0; h < cnt[s]; ++h) {
            long long inc = 0, esc = 0;
            replay_history<false, false, false, true>(a, sp, pl, lut.data(), wc, h, 0, inc, esc, sink, work);
            incident += inc;
            escaped += esc;
            // the same history once more for its end point
            a.ep_xyz = xyz;
            a.ep_reason = &reason;
            long long i2 = 0, e2_ = 0;
            WorkCount none{0u, 0u, 0u};
            replay_history<true, false, false, false>(a, sp, pl, lut.data(), wc, h, 0, i2, e2_, NullSink{}, none);
            a.ep_xyz = nullptr;
            a.ep_reason = nullptr;
            ep_xyz.insert(ep_xyz.end(), xyz, xyz + 3);
            ep_reason.push_back(reason);
        }
    }
    const std::string pre = argv[3];
    FILE *o = std::fopen((pre + ".E").c_str(), "wb");
    std::fwrite(E.data(), 8, nvox, o);
    std::fclose(o);
    o = std::fopen((pre + ".E2").c_str(), "wb");
    std::fwrite(E2.data(), 8, nvox, o);
    std::fclose(o);
    o = std::fopen((pre + ".ep").c_str(), "wb");
    for (size_t i = 0; i < ep_reason.size(); ++i) {
        std::fwrite(&ep_xyz[3 * i], 4, 3, o);
        std::fwrite(&ep_reason[i], 4, 1, o);
    }
    std::fclose(o);
    std::printf("%lld %lld %u %u %u\n", incident, escaped, work.steps, work.visits, work.flushes);
    return 0;
}
