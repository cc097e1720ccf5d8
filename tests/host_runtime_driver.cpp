// Drives the library's host runtime through a context without a GPU
// (FDC_NO_DEVICE) for sanitizer builds: every argument check, the loaders'
// validation, the database file reader, the plan and spot bookkeeping, the
// overflow guard and the launch-config rules.  Prints "ok" and exits 0 when
// every status code is the documented one.  Usage: host_runtime_driver db.bin
#include "fdc.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int failures = 0;

static void expect(int got, int want, const char *what)
{
    if (got != want) {
        std::printf("FAIL %s: got %d, want %d\n", what, got, want);
        ++failures;
    }
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    fdc_ctx *c = nullptr;
    expect(fdc_create(nullptr, FDC_NO_DEVICE, 1, 64), FDC_E_ARG, "create NULL");
    expect(fdc_create(&c, FDC_NO_DEVICE, 1, 0), FDC_E_ARG, "create R=0");
    expect(fdc_create(&c, FDC_NO_DEVICE, 1, 64), FDC_OK, "create");
    if (!c) return 1;

    const float hu[4] = {-1000.f, 0.f, 1000.f, 3071.f}, rho[4] = {0.0012f, 1.f, 1.6f, 2.84f};
    const float rsp[4] = {0.0011f, 1.f, 1.5f, 2.64f}, rscp[4] = {0.0012f, 1.f, 2.16f, 3.834f};
    expect(fdc_set_hu_table(c, hu, rho, rsp, rscp, 4, -990.f), FDC_OK, "table");
    expect(fdc_set_hu_table(c, hu, rho, rsp, rscp, 1, -990.f), FDC_E_ARG, "table n=1");
    const float bad_hu[4] = {-1000.f, 0.f, 0.f, 3071.f};
    expect(fdc_set_hu_table(c, bad_hu, rho, rsp, rscp, 4, -990.f), FDC_E_ARG, "table order");

    // a database of two bins x two tracks x three steps
    std::vector<fdc_step> steps(12, fdc_step{0.1f, 1.0f, 0.002f, 0.3f});
    const uint64_t off[5] = {0, 3, 6, 9, 12};
    const float bin_E[2] = {3.0f, 3.5f};
    const uint32_t bin_first[3] = {0, 2, 4};
    expect(fdc_add_beam_spots(c, 0, nullptr, 0), FDC_E_ARG, "spots before any plan");
    expect(fdc_load_track_db(c, steps.data(), 12, off, 4, bin_E, bin_first, 2, nullptr), FDC_OK, "db");
    const uint64_t bad_off[5] = {0, 3, 3, 9, 12};
    expect(fdc_load_track_db(c, steps.data(), 12, bad_off, 4, bin_E, bin_first, 2, nullptr), FDC_E_FORMAT, "db offsets");
    steps[5].dx_cm = NAN;
    expect(fdc_load_track_db(c, steps.data(), 12, off, 4, bin_E, bin_first, 2, nullptr), FDC_E_FORMAT, "db NaN");
    steps[5].dx_cm = 0.1f;
    expect(fdc_load_track_db_file(c, argv[1], nullptr), FDC_OK, "db file");
    expect(fdc_load_track_db_file(c, "/nonexistent/db.bin", nullptr), FDC_E_ARG, "db file missing");
    expect(fdc_load_track_db_file(c, nullptr, nullptr), FDC_E_ARG, "db file NULL");

    std::vector<int16_t> ph(6 * 5 * 4, 0);
    const float vox[3] = {0.5f, 0.5f, 0.5f}, org[3] = {-1.5f, -1.25f, 0.f};
    int32_t plan = -1;
    expect(fdc_load_phantom(c, &plan, ph.data(), 6, 5, 4, vox, org, nullptr), FDC_OK, "phantom");
    expect(plan, 0, "plan id");
    const float bad_vox[3] = {0.5f, 0.f, 0.5f};
    expect(fdc_load_phantom(c, &plan, ph.data(), 6, 5, 4, bad_vox, org, nullptr), FDC_E_ARG, "phantom voxel 0");
    expect(fdc_load_phantom(c, &plan, ph.data(), 0, 5, 4, vox, org, nullptr), FDC_E_ARG, "phantom nx 0");
    expect(plan, 0, "plan id kept");

    // spot energies must lie within the bins of the database now loaded (from the file)
    fdc_spot s{};
    s.pos_cm[2] = -1.f;
    s.dir[2] = 1.f;
    s.sigma_cm = 0.2f;
    s.n_histories = 1000;
    s.energy_MeV = 1.0e6f;
    expect(fdc_add_beam_spots(c, plan, &s, 1), FDC_E_RANGE, "spot above bins");
    s.energy_MeV = NAN;
    expect(fdc_add_beam_spots(c, plan, &s, 1), FDC_E_ARG, "spot NaN");
    std::printf("last error: %s\n", fdc_last_error(c));
    expect(fdc_add_beam_spots(c, 7, &s, 1), FDC_E_ARG, "spot bad plan");

    expect(fdc_load_track_db(c, steps.data(), 12, off, 4, bin_E, bin_first, 2, nullptr), FDC_OK, "db again");
    s.energy_MeV = 3.2f;
    expect(fdc_add_beam_spots(c, plan, &s, 1), FDC_OK, "spot");
    const int32_t plans[2] = {0, 0};
    expect(fdc_run_histories(c, plans, 2, FDC_RUN_VARIANCE, nullptr), FDC_E_ARG, "run duplicate plan");
    expect(fdc_run_histories(c, plans, 1, 64u, nullptr), FDC_E_ARG, "run flag");
    expect(fdc_run_histories(c, plans, 1, FDC_RUN_VARIANCE, nullptr), FDC_OK, "run");
    fdc_summary sum;
    expect(fdc_read_dose_and_variance(c, 0, nullptr, nullptr, nullptr, nullptr, &sum, nullptr), FDC_E_STATE,
           "read without a device");
    fdc_graph *g = nullptr;
    expect(fdc_graph_create(c, plans, 1, FDC_RUN_VARIANCE, 0, nullptr, nullptr, &g), FDC_E_STATE, "graph dry");
    s.n_histories = 4000000000000000ull;
    expect(fdc_add_beam_spots(c, plan, &s, 1), FDC_OK, "huge spot");
    expect(fdc_run_histories(c, plans, 1, 0, nullptr), FDC_E_OVERFLOW, "overflow guard");
    expect(fdc_reset_plan(c, 0, 1, nullptr), FDC_OK, "reset");

    fdc_launch_config cfg{};
    cfg.waves_per_block = 16;
    cfg.blocks_per_cu = 1;
    cfg.tally_slots = 8064;
    cfg.units_per_wave = 1;
    cfg.tally_mode = 2;
    cfg.source_order = 1;
    expect(fdc_set_launch_config(c, &cfg), FDC_OK, "launch config");
    cfg.tally_slots = 8100;
    expect(fdc_set_launch_config(c, &cfg), FDC_E_ARG, "launch config slots");
    cfg.waves_per_block = 17;
    expect(fdc_set_launch_config(c, &cfg), FDC_E_ARG, "launch config waves");

    expect(fdc_destroy(c), FDC_OK, "destroy");
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
