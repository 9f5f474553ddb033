// sad_host.h -- host-side validation and error reporting shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "sad.h"

namespace sad {

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Check the image descriptor; fills the effective score scale.
inline sad_status check_image(const sad_image *img, float *s_eff) {
    if (!img) {
        set_error("image descriptor is NULL");
        return SAD_ERR_INVALID_ARGUMENT;
    }
    if (img->H <= 0 || img->W <= 0 || (int64_t)img->H * img->W > (int64_t)1 << 30) {
        set_error("bad image size %d x %d", img->H, img->W);
        return SAD_ERR_INVALID_ARGUMENT;
    }
    if (img->K < 4 || img->K > SAD_MAX_K || (img->K & 3)) {
        set_error("K = %d unsupported (multiple of 4 in [4, %d])", img->K, SAD_MAX_K);
        return SAD_ERR_UNSUPPORTED;
    }
    if (img->n_slots < 0 || img->cap < img->n_slots || img->cap > ((int64_t)1 << 31)) {
        set_error("bad slot counts n_slots = %d, cap = %lld", img->n_slots, (long long)img->cap);
        return SAD_ERR_INVALID_ARGUMENT;
    }
    float s = img->score_scale;
    if (s == 0.0f) s = 1.0f / (float)(img->H > img->W ? img->H : img->W);
    if (!(s > 0.0f) || s != s || s > 3.0e38f) {
        set_error("bad score scale %g", (double)img->score_scale);
        return SAD_ERR_INVALID_ARGUMENT;
    }
    if (s_eff) *s_eff = s;
    return SAD_OK;
}

inline sad_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return SAD_ERR_DEVICE;
    }
    return SAD_OK;
}

#define SAD_REQUIRE(cond, code, ...)  \
    do {                              \
        if (!(cond)) {                \
            ::sad::set_error(__VA_ARGS__); \
            return code;              \
        }                             \
    } while (0)

#define SAD_TRY(expr)                     \
    do {                                  \
        sad_status _st = (expr);          \
        if (_st != SAD_OK) return _st;    \
    } while (0)

// Number of 16x16 tiles.
inline int tiles_x(const sad_image *img) { return (img->W + 15) / 16; }
inline int n_tiles(const sad_image *img) { return tiles_x(img) * ((img->H + 15) / 16); }

}  // namespace sad
