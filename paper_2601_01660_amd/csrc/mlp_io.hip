// Checkpoint of a learned per-light transmittance field: parameters, optional
// Adam moments and the step count, with the atlas geometry the features were
// built for (the Fourier frequencies depend on the atlas width).
//
// File layout: a first line "DGSM-MLP 1", a second line holding a JSON object
// {"params": P, "adam": 0|1, "step": t, "H": .., "W": .., "K": .., "spacing": ..,
//  "r0": .., "r1": ..}, then P float32 values (little endian) and, with adam = 1,
// 2 P more (first moments, then second moments).  Host code only.

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "dgsm.h"
#include "mlp.hpp"

namespace {

constexpr const char* kMagic = "DGSM-MLP 1";

// Value of "key" in a flat JSON object of numbers, or false if absent.
bool json_number(const std::string& js, const char* key, double& out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = js.find(k);
    if (at == std::string::npos) return false;
    size_t c = js.find(':', at + k.size());
    if (c == std::string::npos) return false;
    const char* p = js.c_str() + c + 1;
    char* end = nullptr;
    out = std::strtod(p, &end);
    return end != p;
}

bool read_line(FILE* f, std::string& line) {
    line.clear();
    for (int ch; (ch = std::fgetc(f)) != EOF;) {
        if (ch == '\n') return true;
        line.push_back((char)ch);
        if (line.size() > 4096) return false;
    }
    return false;
}

}  // namespace

extern "C" dgsm_status dgsm_mlp_save(const char* path, const float* params, const float* adam_mv, int32_t step,
                                     const dgsm_atlas_desc_t* desc) {
    if (!path || !params || !desc || step < 0) return DGSM_EINVAL;
    FILE* f = std::fopen(path, "wb");
    if (!f) return DGSM_EINVAL;
    const int P = dgsm::mlp::kNParams;
    char head[512];
    std::snprintf(head, sizeof head,
                  "%s\n{\"params\": %d, \"adam\": %d, \"step\": %d, \"H\": %d, \"W\": %d, \"K\": %d, "
                  "\"spacing\": %d, \"r0\": %.9g, \"r1\": %.9g}\n",
                  kMagic, P, adam_mv ? 1 : 0, step, desc->H, desc->W, desc->K, desc->spacing, (double)desc->r0,
                  (double)desc->r1);
    bool ok = std::fputs(head, f) >= 0 && std::fwrite(params, sizeof(float), P, f) == (size_t)P;
    if (ok && adam_mv) ok = std::fwrite(adam_mv, sizeof(float), 2 * (size_t)P, f) == 2 * (size_t)P;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? DGSM_OK : DGSM_EINVAL;
}

extern "C" dgsm_status dgsm_mlp_load(const char* path, float* params, float* adam_mv, int32_t* step,
                                     dgsm_atlas_desc_t* desc) {
    if (!path || !params) return DGSM_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return DGSM_EINVAL;
    std::string magic, js;
    double np = 0, adam = 0, st = 0, H = 0, W = 0, K = 0, sp = 0, r0 = 0, r1 = 0;
    bool ok = read_line(f, magic) && magic == kMagic && read_line(f, js) && json_number(js, "params", np) &&
              json_number(js, "adam", adam) && json_number(js, "step", st) && json_number(js, "H", H) &&
              json_number(js, "W", W) && json_number(js, "K", K) && json_number(js, "spacing", sp) &&
              json_number(js, "r0", r0) && json_number(js, "r1", r1) && (int)np == dgsm::mlp::kNParams &&
              !(adam_mv && adam == 0);
    const int P = dgsm::mlp::kNParams;
    ok = ok && std::fread(params, sizeof(float), P, f) == (size_t)P;
    if (ok && adam_mv) ok = std::fread(adam_mv, sizeof(float), 2 * (size_t)P, f) == 2 * (size_t)P;
    std::fclose(f);
    if (!ok) return DGSM_EINVAL;
    if (step) *step = (int32_t)st;
    if (desc) {
        std::memset(desc, 0, sizeof *desc);
        desc->H = (int32_t)H;
        desc->W = (int32_t)W;
        desc->K = (int32_t)K;
        desc->spacing = (int32_t)sp;
        desc->r0 = (float)r0;
        desc->r1 = (float)r1;
        desc->param = DGSM_PARAM_OCTAHEDRAL;
    }
    return DGSM_OK;
}
