// tune.hip -- tile-shape tables of the forward filter and the batch kernels,
// and the per-image autotuner.
//
// The per-image table maps (window, kind, dist, input type) to one of the
// extended-tile shapes of odf_internal.h; the batch table maps each batch
// group (window 3 / 5 x BVDF / DDF) to one.  odf_autotune times every valid
// shape on a seeded tuning image with HIP events, keeps the fastest and
// records the timings in a small JSON cache keyed by the GPU architecture
// (odf_autotune_batch, in batch.hip, does the same for a batch group);
// odf_tune_load reads such a cache back.  The tables are process-wide;
// updates are atomic per entry.
#include <atomic>
#include <math.h>
#include <mutex>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "odf.h"
#include "odf_internal.h"

namespace odf {

namespace {

// [window 3/5/7][kind ODF_BVDF .. ODF_CWDDF][dist][u8]
constexpr int kTableKinds = 5;
std::atomic<int> g_table[4][kTableKinds][3][2];
std::once_flag g_table_once;

int window_slot(int window) { return (window - 3) / 2; }  // 3, 5, 7, 9

// The centre-weighted vector median has no angular term: its kernel runs the
// chromaticity layout whatever dist the caller names, so every dist shares
// one entry.
int dist_slot(int kind, int dist) { return kind == ODF_CWVMF ? (int)kRgb : dist; }

// Batch groups: 32 x 32 for 3x3 DDF and 32 x 16 otherwise until tuned (the
// steady-state best measured on MI355X on 3840 x 2160 frames).
std::atomic<int> g_batch[kNumBatchGroups];

void ensure_init() {
    std::call_once(g_table_once, [] {
        for (int w = 0; w < 4; ++w)
            for (int k = 0; k < kTableKinds; ++k)
                for (int d = 0; d < 3; ++d)
                    for (int u = 0; u < 2; ++u)
                        g_table[w][k][d][u].store(tile_config_default(3 + 2 * w, k));
        for (int g = 0; g < kNumBatchGroups; ++g) g_batch[g].store(g == 1 ? 0 : 2);
    });
}

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): seeded numbers for the tuning images
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double unit(uint64_t& s) { return (double)(splitmix(s) >> 11) * 0x1p-53; }

}  // namespace

int batch_tuned_config(int group) {
    ensure_init();
    return g_batch[group].load();
}

void set_batch_tuned_config(int group, int cfg) {
    ensure_init();
    g_batch[group].store(cfg);
}

void tuning_image(int M, int N, uint64_t seed, uint8_t* out) {
    uint64_t s = seed;
    double a[3][4], fx[3][4], fy[3][4], ph[3][4];
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 4; ++j) {
            const double f = (1.0 / 96.0) + unit(s) * (1.0 / 24.0), th = unit(s) * 3.14159265;
            a[k][j] = 0.5 + 0.5 * unit(s);
            fx[k][j] = f * cos(th);
            fy[k][j] = f * sin(th);
            ph[k][j] = unit(s) * 6.28318531;
        }
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < N; ++c) {
            uint8_t* px = out + ((size_t)r * N + c) * 3;
            if (unit(s) < 0.15) {  // impulsive noise: a random colour
                const uint64_t v = splitmix(s);
                px[0] = (uint8_t)v; px[1] = (uint8_t)(v >> 8); px[2] = (uint8_t)(v >> 16);
                continue;
            }
            for (int k = 0; k < 3; ++k) {
                double v = 0.0, n = 0.0;
                for (int j = 0; j < 4; ++j) {
                    v += a[k][j] * sin(6.28318531 * (fx[k][j] * c + fy[k][j] * r) + ph[k][j]);
                    n += a[k][j];
                }
                px[k] = (uint8_t)lrint(127.5 + 127.5 * v / n);
            }
        }
}

// kind: the C ABI's odf_kind (ODF_BVDF .. ODF_CWDDF)
int tuned_config(int window, int kind, int dist, bool u8) {
    ensure_init();
    return g_table[window_slot(window)][kind][dist_slot(kind, dist)][u8 ? 1 : 0].load();
}

void set_tuned_config(int window, int kind, int dist, bool u8, int cfg) {
    ensure_init();
    g_table[window_slot(window)][kind][dist_slot(kind, dist)][u8 ? 1 : 0].store(cfg);
}

// The kernel family of a C ABI kind.
int kernel_kind(int kind) {
    switch (kind) {
    case ODF_ACWDDF: return kACW;
    case ODF_CWVMF: return kCWV;
    case ODF_CWDDF: return kCW;
    default: return kind;  // ODF_BVDF, ODF_DDF
    }
}

}  // namespace odf

namespace {

// A (window, kind, dist) class the library computes (the centre-weighted
// kinds have no 7x7 or 9x9 kernels).
bool valid_class(int window, int kind, int dist) {
    if (window != 3 && window != 5 && window != 7 && window != 9) return false;
    if (kind < ODF_BVDF || kind > ODF_CWDDF) return false;
    if (window == 9 && kind != ODF_BVDF && kind != ODF_DDF) return false;
    return dist >= 0 && dist <= 2;
}

}  // namespace

extern "C" {

int odf_tile_config(int config, int* ext_w, int* ext_h) {
    if (config < 0 || config >= odf::kNumTileConfigs || !ext_w || !ext_h) return ODF_EINVAL;
    odf::tile_config_shape(config, ext_w, ext_h);
    return ODF_OK;
}

int odf_tune_get(int window, int kind, int dist, int is_u8) {
    if (!valid_class(window, kind, dist)) return ODF_EINVAL;
    return odf::tuned_config(window, kind, dist, is_u8 != 0);
}

int odf_tune_set(int window, int kind, int dist, int is_u8, int config) {
    if (!valid_class(window, kind, dist) ||
        !odf::tile_config_valid(window, odf::kernel_kind(kind), config, is_u8 != 0))
        return ODF_EINVAL;
    odf::set_tuned_config(window, kind, dist, is_u8 != 0, config);
    return ODF_OK;
}

int odf_autotune(int window, int kind, int dist, int is_u8, int M, int N, int reps,
                 const char* cache_path, float* times_ms, void* stream) {
    if (!valid_class(window, kind, dist) || M < 1 || N < 1 || reps < 1 ||
        (long long)M * N >= (1ll << 28))
        return odf::set_error(ODF_EINVAL, "autotune: arguments out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int kk = odf::kernel_kind(kind);
    const int kd = kind == ODF_CWVMF ? ODF_RGB : dist;  // the kernel's pair term
    const size_t npix = (size_t)M * N;
    const size_t esz = is_u8 ? 1 : 4;
    std::vector<uint8_t> h8;
    std::vector<float> hf;
    try {  // no exception crosses the C ABI
        h8.resize(npix * 3);
        hf.resize(is_u8 ? 0 : npix * 3);
    } catch (...) {
        return odf::set_error(ODF_ENOMEM, "autotune: host allocation failed");
    }
    odf::tuning_image(M, N, 1009, h8.data());
    if (!is_u8)
        for (size_t i = 0; i < npix * 3; ++i) hf[i] = h8[i] / 255.0f;
    void *img = nullptr, *out = nullptr;
    uint8_t* idx = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ODF_OK;
    int best = -1;
    float best_ms = 0.0f;
    float ms_all[odf::kNumTileConfigs];
    if (odf::test_fail_alloc() || hipMalloc(&img, npix * 3 * esz) != hipSuccess ||
        hipMalloc(&out, npix * 3 * esz) != hipSuccess || hipMalloc(&idx, npix) != hipSuccess) {
        rc = odf::set_error(ODF_ENOMEM, "autotune: device allocation failed");
        goto done;
    }
    if (hipMemcpy(img, is_u8 ? (const void*)h8.data() : (const void*)hf.data(), npix * 3 * esz,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = ODF_EHIP;
        goto done;
    }
    for (int cfg = 0; cfg < odf::kNumTileConfigs; ++cfg) {
        ms_all[cfg] = -1.0f;
        if (!odf::tile_config_valid(window, kk, cfg, is_u8 != 0)) continue;
        odf::FwdParams prm{};
        prm.img = img; prm.out = out; prm.idx = idx;
        prm.B = 1; prm.M = M; prm.N = N;
        prm.p = kind == ODF_DDF ? 0.25f : (kind == ODF_BVDF ? 0.0f : 0.5f);
        if (kd == ODF_MINIMAX) prm.coef = odf::minimax_coef(4);  // timing does not depend on q
        if (kind == ODF_ACWDDF) odf::set_acw_params(window, 2, 10.8f, prm);
        if (kind == ODF_CWVMF || kind == ODF_CWDDF)  // level 2: centre weight n - 2
            for (int j = 0; j < 3; ++j) prm.acw_wm1[j] = (float)(window * window - 3);
        for (int w = 0; w < 2; ++w)
            if (odf::launch_forward(window, kk, kd, is_u8 != 0, false, cfg, prm, s) != hipSuccess) {
                rc = ODF_EHIP;
                goto done;
            }
        bool ok = hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; r < reps; ++r)
            ok = ok && odf::launch_forward(window, kk, kd, is_u8 != 0, false, cfg, prm, s) ==
                           hipSuccess;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = ODF_EHIP;
            goto done;
        }
        ms /= reps;
        ms_all[cfg] = ms;
        if (best < 0 || ms < best_ms) {
            best = cfg;
            best_ms = ms;
        }
    }
    if (best >= 0) odf::set_tuned_config(window, kind, dist, is_u8 != 0, best);
    if (times_ms)
        for (int c = 0; c < odf::kNumTileConfigs; ++c) times_ms[c] = ms_all[c];
    if (cache_path && best >= 0) {
        hipDeviceProp_t prop;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            rc = ODF_EHIP;
            goto done;
        }
        FILE* f = fopen(cache_path, "a");
        if (!f) {
            rc = odf::set_error(ODF_EINVAL, "cannot open %s", cache_path);
            goto done;
        }
        fprintf(f,
                "{\"arch\": \"%s\", \"window\": %d, \"kind\": %d, \"dist\": %d, \"u8\": %d, "
                "\"config\": %d, \"M\": %d, \"N\": %d, \"ms\": [%.5f, %.5f, %.5f, %.5f, %.5f, "
                "%.5f]}\n",
                prop.gcnArchName, window, kind, dist, is_u8 != 0, best, M, N, ms_all[0],
                ms_all[1], ms_all[2], ms_all[3], ms_all[4], ms_all[5]);
        fclose(f);
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (img) (void)hipFree(img);
    if (out) (void)hipFree(out);
    if (idx) (void)hipFree(idx);
    return best >= 0 || rc != ODF_OK ? rc : ODF_EHIP;
}

int odf_batch_tune_get(int window, int kind) {
    if (!odf::batch_window(window) || (kind != ODF_BVDF && kind != ODF_DDF)) return ODF_EINVAL;
    return odf::batch_tuned_config(odf::batch_group(window, kind));
}

int odf_batch_tune_set(int window, int kind, int config) {
    if (!odf::batch_window(window) || (kind != ODF_BVDF && kind != ODF_DDF) ||
        !odf::tile_config_valid(window, kind, config, true))
        return ODF_EINVAL;
    odf::set_batch_tuned_config(odf::batch_group(window, kind), config);
    return ODF_OK;
}

int odf_tune_load(const char* cache_path) {
    if (!cache_path) return ODF_EINVAL;
    FILE* f = fopen(cache_path, "r");
    if (!f) return ODF_EINVAL;
    hipDeviceProp_t prop;
    int dev = 0;
    const bool have_dev =
        hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess;
    char line[512];
    int applied = 0;
    while (fgets(line, sizeof line, f)) {
        char arch[128] = "";
        int w, k, d, u, c;
        if (sscanf(line,
                   "{\"arch\": \"%127[^\"]\", \"window\": %d, \"kind\": %d, \"dist\": %d, "
                   "\"u8\": %d, \"config\": %d",
                   arch, &w, &k, &d, &u, &c) == 6) {
            if (have_dev && strcmp(arch, prop.gcnArchName) != 0) continue;
            if (odf_tune_set(w, k, d, u, c) == ODF_OK) ++applied;
        } else if (sscanf(line,
                          "{\"arch\": \"%127[^\"]\", \"batch_window\": %d, \"kind\": %d, "
                          "\"config\": %d",
                          arch, &w, &k, &c) == 4) {
            if (have_dev && strcmp(arch, prop.gcnArchName) != 0) continue;
            if (odf_batch_tune_set(w, k, c) == ODF_OK) ++applied;
        }  // other lines are ignored
    }
    fclose(f);
    return applied;
}

}  // extern "C"
