// Host-side checks of libnb built with AddressSanitizer and UBSan on its host
// code (tests/test_sanitizers.py): every entry point that needs no GPU --
// status strings, parameter validation and arena sizing over the parameter
// space, and the error paths of calls given NULL handles.  Exit status 0 when
// every call returned what the ABI documents.
#include <cstdio>
#include <cstring>

#include "../include/nb.h"

static int failures = 0;

static void expect(bool ok, const char* what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

static nb_params base_params()
{
    nb_params p;
    std::memset(&p, 0, sizeof(p));
    p.n_atoms = 3000;
    p.box[0] = 3.0;
    p.box[1] = 3.1;
    p.box[2] = 3.2;
    p.r_cut = 0.9;
    p.r_list = 1.0;
    p.coulomb = NB_COUL_EWALD;
    p.eps_r = 1.0;
    p.ewald_beta = 3.12;
    p.lj = NB_LJ_SINGLE;
    p.c6 = 2.6e-3;
    p.c12 = 2.6e-6;
    p.flags = NB_POT_SHIFT;
    return p;
}

int main()
{
    for (int c = -12; c <= 2; ++c) expect(nb_strerror((nb_status)c) != nullptr, "nb_strerror");
    size_t bytes = 0;
    // valid systems across cluster sizes, models, boxes, pruning and PME
    const int clusters[] = {0, 1, 4, 8};
    for (int cl : clusters)
        for (int coul = 0; coul <= 2; ++coul)
            for (int lj = 0; lj <= 1; ++lj) {
                nb_params p = base_params();
                p.cluster = cl;
                p.coulomb = coul;
                p.lj = lj;
                expect(nb_arena_bytes(&p, &bytes) == NB_OK && bytes > 0, "valid model");
            }
    {
        nb_params p = base_params();
        p.box[2] = 3.0 / 1.4142135623730951;
        p.box[0] = p.box[1] = 3.0;
        p.box_off[1] = p.box_off[2] = 1.5;  // rhombic dodecahedron
        expect(nb_arena_bytes(&p, &bytes) == NB_OK, "dodecahedron");
        p.r_inner = 0.95;
        p.nstprune = 4;
        expect(nb_arena_bytes(&p, &bytes) == NB_OK, "pruning");
        p.pme_grid[0] = 24;
        p.pme_grid[1] = 24;
        p.pme_grid[2] = 17;
        p.pme_order = 6;
        expect(nb_arena_bytes(&p, &bytes) == NB_OK, "PME");
    }
    {
        nb_params p = base_params();
        p.n_atoms = 1;
        expect(nb_arena_bytes(&p, &bytes) == NB_OK, "one atom");
        p.n_atoms = 2000000;
        p.box[0] = p.box[1] = p.box[2] = 27.0;
        expect(nb_arena_bytes(&p, &bytes) == NB_OK && bytes > ((size_t)1 << 30), "two million atoms");
    }
    // invalid parameters: each is refused with the documented code
    struct Bad {
        const char* what;
        void (*edit)(nb_params&);
        nb_status code;
    };
    const Bad bad[] = {
        {"no atoms", [](nb_params& p) { p.n_atoms = 0; }, NB_ERR_ARG},
        {"negative box", [](nb_params& p) { p.box[1] = -1.0; }, NB_ERR_BOX},
        {"r_list beyond half the box", [](nb_params& p) { p.r_list = 1.6; }, NB_ERR_BOX},
        {"r_cut above r_list", [](nb_params& p) { p.r_cut = 1.1; }, NB_ERR_ARG},
        {"coulomb kind", [](nb_params& p) { p.coulomb = 7; }, NB_ERR_ARG},
        {"cluster size", [](nb_params& p) { p.cluster = 3; }, NB_ERR_ARG},
        {"skew beyond half an edge", [](nb_params& p) { p.box_off[0] = 1.6; }, NB_ERR_BOX},
        {"r_inner below r_cut", [](nb_params& p) { p.r_inner = 0.5; p.nstprune = 2; }, NB_ERR_ARG},
        {"PME grid below the order", [](nb_params& p) { p.pme_grid[0] = p.pme_grid[1] = p.pme_grid[2] = 3; }, NB_ERR_ARG},
        {"PME grid above 256", [](nb_params& p) { p.pme_grid[0] = p.pme_grid[1] = p.pme_grid[2] = 300; }, NB_ERR_ARG},
        {"PME without Ewald", [](nb_params& p) { p.coulomb = NB_COUL_RF; p.pme_grid[0] = p.pme_grid[1] = p.pme_grid[2] = 24; }, NB_ERR_ARG},
        {"unknown flag", [](nb_params& p) { p.flags = 0x80; }, NB_ERR_ARG},
    };
    for (const Bad& b : bad) {
        nb_params p = base_params();
        b.edit(p);
        expect(nb_arena_bytes(&p, &bytes) == b.code, b.what);
        expect(nb_last_error(nullptr) != nullptr && std::strlen(nb_last_error(nullptr)) > 0, "message");
    }
    expect(nb_arena_bytes(nullptr, &bytes) == NB_ERR_ARG, "NULL params");
    // NULL handles
    expect(nb_sys_destroy(nullptr) == NB_ERR_ARG, "destroy NULL");
    expect(nb_ctx_destroy(nullptr) == NB_ERR_ARG, "ctx destroy NULL");
    expect(nb_build_pairlist(nullptr, nullptr) == NB_ERR_ARG, "build NULL");
    expect(nb_compute_forces(nullptr, nullptr, nullptr, nullptr, nullptr) == NB_ERR_ARG, "forces NULL");
    expect(nb_pme_forces(nullptr, nullptr, nullptr, nullptr, nullptr) == NB_ERR_ARG, "pme NULL");
    std::printf("host driver: %d failure(s)\n", failures);
    return failures == 0 ? 0 : 1;
}
