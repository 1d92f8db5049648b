// Host-only driver of the library's argument validation and checkpoint I/O,
// built with the address and undefined-behaviour sanitizers on the host code
// (tests/test_abi.py builds and runs it; no GPU is touched).  Every call below
// must return before any device work: invalid descriptions, null or fake
// device pointers, short workspaces, malformed checkpoint files.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dgsm.h"

static int failures = 0;

#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                               \
        }                                                             \
    } while (0)

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : ".";
    void* fake = reinterpret_cast<void*>(uintptr_t(1) << 40);   // never dereferenced on the host
    const float* ff = static_cast<const float*>(fake);
    for (int s = 0; s < 8; ++s) EXPECT(dgsm_status_string((dgsm_status)s) != nullptr);   // 5..7: unknown

    dgsm_atlas_desc_t d{};
    d.H = 32; d.W = 32; d.K = 16; d.spacing = DGSM_SHELLS_GEOMETRIC; d.r0 = 0.05f; d.r1 = 8.f;
    d.dtype = DGSM_F32; d.cull_eps = 1e-8f; d.param = DGSM_PARAM_OCTAHEDRAL;
    EXPECT(dgsm_build_workspace_size(&d, 1000, 2) > 0);
    EXPECT(dgsm_build_workspace_size(nullptr, 1000, 2) == 0);
    EXPECT(dgsm_build_workspace_size(&d, -1, 2) == 0);
    EXPECT(dgsm_build_workspace_size(&d, 1000, 0) == 0);
    EXPECT(dgsm_build_workspace_size_entries(&d, 1000, 2, 0) > 0);
    EXPECT(dgsm_build_workspace_size_entries(&d, 1000, 2, 0) <= dgsm_build_workspace_size(&d, 1000, 2));
    EXPECT(dgsm_build_workspace_size_entries(&d, 1000, 2, -5) == 0);
    EXPECT(dgsm_build_workspace_size_entries(&d, 1000, 2, int64_t(1) << 40) == dgsm_build_workspace_size(&d, 1000, 2));
    dgsm_atlas_desc_t bad[6] = {d, d, d, d, d, d};
    bad[0].H = 3; bad[1].K = 1; bad[2].r0 = 9.f; bad[3].dtype = 7; bad[4].param = 9; bad[5].H = 4096;
    for (auto& b : bad) EXPECT(dgsm_build_workspace_size(&b, 10, 1) == 0);

    dgsm_lights_t L{ff, 2, 1.f, 0};
    dgsm_gaussians_t G{ff, ff, ff, ff, 1000};
    const size_t ws = dgsm_build_workspace_size(&d, 1000, 2);
    EXPECT(dgsm_build(nullptr, &G, &d, fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build(&L, nullptr, &d, fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build(&L, &G, &bad[0], fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build(&L, &G, &d, nullptr, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build(&L, &G, &d, fake, nullptr, ws, nullptr) == DGSM_EWORKSPACE);
    EXPECT(dgsm_build(&L, &G, &d, fake, fake, 100, nullptr) == DGSM_EWORKSPACE);
    dgsm_lights_t L0{ff, 0, 1.f, 0}, Lb{ff, 1, 1.f, 9};
    EXPECT(dgsm_build(&L0, &G, &d, fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build(&Lb, &G, &d, fake, fake, ws, nullptr) == DGSM_EINVAL);
    dgsm_gaussians_t Gn{ff, ff, ff, ff, -1};
    EXPECT(dgsm_build(&L, &Gn, &d, fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_bin(&L, &G, &d, fake, 100, nullptr) == DGSM_EWORKSPACE);
    EXPECT(dgsm_accumulate(&L, &d, 1000, fake, fake, 100, nullptr, nullptr) == DGSM_EWORKSPACE);
    dgsm_accum_opts_t ao{3, 0, 0};
    EXPECT(dgsm_accumulate_ex(&L, &d, 1000, fake, fake, ws, &ao, nullptr, nullptr) == DGSM_EINVAL);
    ao = {8, 0, 1};
    EXPECT(dgsm_accumulate_ex(&L, &d, 1000, fake, fake, ws, &ao, static_cast<unsigned long long*>(fake), nullptr) ==
           DGSM_EINVAL);
    int64_t ent = 0, le[2];
    EXPECT(dgsm_count_entries(&L, &G, &d, fake, 100, &ent, nullptr) == DGSM_EWORKSPACE);
    EXPECT(dgsm_count_entries(&L, &G, &d, fake, ws, nullptr, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_list_entries(&d, 1000, 2, fake, ws, 2, le, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_query(&L, &bad[1], fake, ff, 10, static_cast<float*>(fake), nullptr) == DGSM_EINVAL);
    dgsm_roi_box_t box{0, 0, 1.f, 2.f, 1.f};   // zmin > zmax
    EXPECT(dgsm_build_roi(&L, &G, &d, ff, 10, &box, fake, fake, ws, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_build_noalloc(&L, &G, &bad[2], fake, nullptr) == DGSM_EINVAL);

    dgsm_plan plan = nullptr;
    int64_t starts[3] = {0, 10, 5};   // not ascending
    dgsm_plan_opts_t po{};
    po.frames = 2; po.static_cache = 1; po.groups = 2; po.group_start = starts;
    EXPECT(dgsm_plan_create(&L, &d, &G, 5, &po, &plan) == DGSM_EINVAL && plan == nullptr);
    po.groups = 1; po.chains = 9;
    EXPECT(dgsm_plan_create(&L, &d, &G, 5, &po, &plan) == DGSM_EINVAL);
    po.chains = 0; po.motion = 5;
    EXPECT(dgsm_plan_create(&L, &d, &G, 5, &po, &plan) == DGSM_EINVAL);
    EXPECT(dgsm_plan_destroy(nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_plan_tile_waves(nullptr) == 0 && dgsm_plan_packed(nullptr) == 0);

    dgsm_sh_params_t sp{32, 64, 1.f, 4.f, 1e-6f, 1.f, ff};
    EXPECT(sh_transfer(ff, 5, &G, nullptr, &sp, static_cast<float*>(fake), nullptr, nullptr, fake, 1 << 20,
                       nullptr) == DGSM_EINVAL);
    EXPECT(sh_transfer(ff, 9, &G, nullptr, &sp, static_cast<float*>(fake), nullptr, nullptr, fake, 16, nullptr) ==
           DGSM_EWORKSPACE);
    EXPECT(sh_transfer(ff, 9, &G, nullptr, &sp, static_cast<float*>(fake), nullptr, nullptr,
                       static_cast<char*>(fake) + 8, 1 << 20, nullptr) == DGSM_EINVAL);
    EXPECT(sh_transfer_workspace_size(32, 64) == 32 * 64 * 16 + 256 + 256 + 256 && sh_transfer_workspace_size(0, 64) == 0);
    EXPECT(dgsm_probe_fit_workspace_size(3) == 0);
    EXPECT(dgsm_mlp_workspace_size(33) == 0);
    EXPECT(dgsm_mlp_check_grid_workspace_size(&d, -1) == 0);
    dgsm_atlas_desc_t cube = d;
    cube.H = 16; cube.W = 24; cube.param = DGSM_PARAM_CUBEMAP;
    EXPECT(dgsm_mlp_check_grid_workspace_size(&cube, 4) == 0);

    // checkpoint I/O (host memory only)
    std::vector<float> p(DGSM_MLP_PARAMS), m(2 * DGSM_MLP_PARAMS), p2(DGSM_MLP_PARAMS), m2(2 * DGSM_MLP_PARAMS);
    for (size_t i = 0; i < p.size(); ++i) p[i] = 0.001f * (float)i - 3.f;
    for (size_t i = 0; i < m.size(); ++i) m[i] = 1e-4f * (float)(i % 977);
    char path[1024];
    std::snprintf(path, sizeof path, "%s/ckpt.dgsm", dir);
    EXPECT(dgsm_mlp_save(path, p.data(), m.data(), 12, &d) == DGSM_OK);
    int32_t step = -1;
    dgsm_atlas_desc_t d2{};
    EXPECT(dgsm_mlp_load(path, p2.data(), m2.data(), &step, &d2) == DGSM_OK);
    EXPECT(step == 12 && d2.H == 32 && d2.W == 32 && d2.K == 16 && d2.r0 == 0.05f);
    EXPECT(std::memcmp(p.data(), p2.data(), p.size() * 4) == 0 && std::memcmp(m.data(), m2.data(), m.size() * 4) == 0);
    // truncated and malformed files
    char path2[1024];
    std::snprintf(path2, sizeof path2, "%s/trunc.dgsm", dir);
    FILE* f = std::fopen(path2, "wb");
    std::fputs("DGSM-MLP 1\n{\"params\": 66177, \"adam\": 1, \"step\": 3, \"H\": 8}\n", f);
    std::fclose(f);
    EXPECT(dgsm_mlp_load(path2, p2.data(), nullptr, nullptr, nullptr) == DGSM_EINVAL);
    f = std::fopen(path2, "wb");
    for (int i = 0; i < 5000; ++i) std::fputc('x', f);   // no newline at all
    std::fclose(f);
    EXPECT(dgsm_mlp_load(path2, p2.data(), nullptr, nullptr, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_mlp_load(nullptr, p2.data(), nullptr, nullptr, nullptr) == DGSM_EINVAL);
    EXPECT(dgsm_mlp_save(path, nullptr, nullptr, 0, &d) == DGSM_EINVAL);

    std::printf("abi_sanitize: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
