// libtg host-side helpers: version, status strings, default parameters.
#include "tg.h"

extern "C" int tg_abi_version(void) { return TG_ABI_VERSION; }

extern "C" const char* tg_status_string(tg_status s) {
    switch (s) {
        case TG_OK: return "ok";
        case TG_ERR_INVALID_ARG: return "invalid argument";
        case TG_ERR_ALIGNMENT: return "misaligned buffer";
        case TG_ERR_WORKSPACE: return "workspace too small";
        case TG_ERR_OVERFLOW: return "capacity overflow";
        case TG_ERR_DEVICE: return "HIP runtime error";
        case TG_ERR_BUDGET: return "request exceeds the memory budget";
        case TG_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

// Renderer constants (the modified 3DGS renderer the paper builds on) and the
// unsolvable thresholds of Sec. 5.2.
extern "C" void tg_default_params(tg_params* p) {
    if (!p) return;
    p->near_z = 0.2f;
    p->dilation = 0.3f;
    p->extent = 3.0f;
    p->j_clamp = 1.3f;
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->t_min = 1e-4f;
    p->static_px = 1.0f;
    p->det_min = 1e-12;
    p->iso_min = 1e-4;
    p->wsum_min = 1e-3;
    p->wsum_total_min = 1e-3;
    p->pix_min = 2;
    p->views_min = 2;
    p->pix_total_min = 3;
    p->coarse_shift = 3;
    p->reg_k = 8;
    p->static_min_pix = 9;
    p->static_frac = 0.9;
    p->static_views = 2;
    p->reserved = 0;
}
