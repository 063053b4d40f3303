// Host-side argument checks of the C ABI, for a build of the library's
// host code with AddressSanitizer and UndefinedBehaviorSanitizer: every
// entry point called with a null context, and the context and tuning
// checks with bad values.  Needs no GPU (a context cannot be created
// without one: CRK_EDEVICE; with one, it is created and destroyed).
// Exits 0 when every status is the documented one.
#include <cstdio>
#include <cstring>

#include "../../include/crk.h"

static int fails = 0;

static void expect(const char *what, int got, int want) {
    if (got != want) {
        std::printf("%s: status %d, expected %d (%s)\n", what, got, want,
                    crk_last_error());
        ++fails;
    }
}

int main() {
    const int E = CRK_EINVAL;
    expect("ctx_create null out", crk_ctx_create(nullptr, CRK_FP32, nullptr, nullptr), E);
    crk_ctx *c = nullptr;
    expect("ctx_create bad precision", crk_ctx_create(&c, 7, nullptr, nullptr), E);
    crk_params bad = {0.5, 1.0, 2.0, 0.01, 1.0};  // gamma <= 1
    expect("ctx_create bad params", crk_ctx_create(&c, CRK_FP32, nullptr, &bad), E);
    const int st = crk_ctx_create(&c, CRK_FP32, nullptr, nullptr);
    if (st == CRK_OK) {
        crk_tuning t;
        expect("get_tuning", crk_get_tuning(c, &t), CRK_OK);
        crk_tuning b = t;
        b.leaf_max = 8;
        expect("tuning leaf_max", crk_set_tuning(c, &b), E);
        b = t;
        b.tile = 3;
        expect("tuning tile", crk_set_tuning(c, &b), E);
        b = t;
        b.sub_sweep = 9;
        expect("tuning sub_sweep", crk_set_tuning(c, &b), E);
        b = t;
        b.act_groups = -1;
        expect("tuning act_groups", crk_set_tuning(c, &b), E);
        expect("density null tree", crk_density(c, nullptr, nullptr, nullptr, nullptr), E);
        expect("graph launch without capture", crk_graph_launch(c), CRK_ESTATE);
        expect("ctx_destroy", crk_ctx_destroy(c), CRK_OK);
    } else {
        expect("ctx_create without a device", st, CRK_EDEVICE);
    }
    expect("set_tuning", crk_set_tuning(nullptr, nullptr), E);
    expect("sync", crk_sync(nullptr, nullptr), E);
    crk_tree *tree = nullptr;
    expect("build_tree", build_tree(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, nullptr, nullptr, &tree), E);
    expect("lists", build_interaction_lists(nullptr, nullptr), E);
    expect("density", crk_density(nullptr, nullptr, nullptr, nullptr, nullptr), E);
    expect("density_noalloc", crk_density_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr), E);
    expect("energy_compatible", crk_hydro_energy_compatible(
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.8, 0.2, 0.01, nullptr,
        nullptr, nullptr), E);
    expect("energy_compatible_block", crk_hydro_energy_compatible_block(
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.8, 0.2, 0.01, 2, nullptr,
        0, nullptr, nullptr, nullptr), E);
    expect("coefficients", crk_coefficients(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), E);
    expect("hydro", crk_hydro_forces(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, nullptr), E);
    expect("gravity", shortrange_gravity(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, nullptr, nullptr), E);
    expect("velocity gradient", crk_velocity_gradient(nullptr, nullptr, nullptr, nullptr, nullptr,
                                                      nullptr, nullptr, nullptr, nullptr,
                                                      nullptr, nullptr), E);
    expect("integrate", crk_integrate(nullptr, 0, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, nullptr), E);
    expect("fof", crk_fof(nullptr, nullptr, 0.1, nullptr, nullptr), E);
    expect("count_pairs", crk_count_pairs(nullptr, nullptr, nullptr), E);
    expect("graph begin", crk_graph_begin(nullptr), E);
    expect("graph end", crk_graph_end(nullptr), E);
    expect("graph launch", crk_graph_launch(nullptr), E);
    expect("graph reset", crk_graph_reset(nullptr), E);
    expect("timing", crk_timing_enable(nullptr, 1), E);
    expect("tree_free", crk_tree_free(nullptr), CRK_OK);
    expect("ctx_destroy", crk_ctx_destroy(nullptr), CRK_OK);
    std::printf("capi driver: %d unexpected statuses\n", fails);
    return fails ? 1 : 0;
}
