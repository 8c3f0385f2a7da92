// internal.h -- host-side internals of libmiaug shared by the C ABI layer and
// the kernel launchers.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/miaug.h"

struct miaug_ctx {
    int device;
    int num_cu;
    int variant;
    int *counters;           // device, 256 ints of queue counters, then kLptMax ints of work order
    std::string arch;        // gcnArchName of the device (tune-cache keys)
    std::string tune_cache;  // autotuner cache file ("" = none)
    miaug_stats stats;
};

namespace miaug {

// ---- runtime.cpp: environment, logging, allocations, tune cache
struct EnvConfig {
    int log_level = 0;
    int force_variant = -1;
    std::string tune_cache;
    long fail_alloc_after = -1;
};
const EnvConfig &env();
// Message to stderr when MIAUG_LOG >= level.
void log_msg(int level, const char *fmt, ...);
// hipMalloc / hipHostMalloc through the failure injector; status as hip_status.
int dev_alloc(void **p, size_t bytes, const char *what);
int pinned_alloc(void **p, size_t bytes, const char *what);
// Arms the injector: the library's allocation number `after` from now fails once (-1 disarms).
void arm_alloc_failure(long after);
struct TuneEntry {
    std::string key, name;
    int variant = -1;
    float ms = 0.f;
};
int tune_cache_read(const std::string &path, std::vector<TuneEntry> &out);
// MIAUG_OK with *hit filled, MIAUG_EUNSUPPORTED when the key is absent.
int tune_cache_get(const std::string &path, const std::string &key, TuneEntry *hit);
int tune_cache_put(const std::string &path, const TuneEntry &e);

// Records a formatted message as the calling thread's last error; returns status.
int set_error(int status, const char *fmt, ...);
// Clears the calling thread's last error (start of every entry point).
void clear_error();
// Maps a HIP error to MIAUG_EDEVICE with context text (MIAUG_OK on success).
int hip_status(hipError_t e, const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---- launchers (each returns the hipError_t of its launches)
hipError_t launch_d4_bc_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const float *ab,
                           uint8_t *out, hipStream_t s);
hipError_t launch_d4_lut_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const uint8_t *luts,
                            const int32_t *gray, uint8_t *out, hipStream_t s);
hipError_t launch_pad_u8(const uint8_t *in, int n, int H, int W, int C, int Ho, int Wo, int border, int value,
                         uint8_t *out, hipStream_t s);
hipError_t launch_warp_u8(const uint8_t *in, int n, int H, int W, int C, const int64_t *aq, int interp, int border,
                          uint8_t *out, hipStream_t s);

constexpr int kLptMax = 4096;  // largest batch the largest-first work order sorts (larger: index order)
struct RaggedLaunch {
    int variant;      // index into the variant table
    int num_cu;       // compute units of the device
    int *counters;    // device: queue counters (8 + 8 padding ints)
    int *order = nullptr;  // device, kLptMax ints: the largest-first work order (NULL: index order)
};
hipError_t launch_ragged(const miaug_ragged_args *a, const RaggedLaunch &L, int per_image, hipStream_t s);
// Row-band form of the batched launch (k_rows.hip); cap_kind 0/1/2 picks the stage size.
hipError_t launch_ragged_rows(const miaug_ragged_args *a, int cap_kind, int wg_per_cu, const RaggedLaunch &L,
                              hipStream_t s);
// Wave-independent row-gather form of the batched launch (k_gather.hip).
hipError_t launch_ragged_gather(const miaug_ragged_args *a, int band, int wg_per_cu, const RaggedLaunch &L,
                                hipStream_t s);
int ragged_variant_count();
bool ragged_variant_enabled(int v);  // false for forms switched off (their names begin "off: ")
const char *ragged_variant_name(int v);
int ragged_default_variant();
// Ints of queue-counter memory launch_ragged uses (RaggedLaunch::counters).
int ragged_counter_ints();

hipError_t launch_c2(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop, int outsz,
                     uint8_t *out, hipStream_t s);
hipError_t launch_c2_mask(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop, int outsz,
                          uint8_t *out, hipStream_t s);
hipError_t launch_blur_u8(const uint8_t *in, int n, int H, int W, int C, int ksize, const int32_t *apply,
                          uint8_t *out, hipStream_t s);
hipError_t launch_hsv_u8(const uint8_t *in, int n, int H, int W, const int32_t *dhsv, uint8_t *out, hipStream_t s);
hipError_t launch_c2_boxes(const float *boxes, const int32_t *box_off, int n, int H, int W,
                           const miaug_c2_record *rec, int crop, int outsz, float *out, hipStream_t s);

hipError_t launch_wc_fwd(const float *x, int n, int C, int H, int W, const float *p, float *y, hipStream_t s);
size_t wc_workspace_bytes(int n, int C, int H, int W);
hipError_t launch_wc_bwd(const float *x, int n, int C, int H, int W, const float *p, const float *gy, float *gx,
                         float *gp, void *ws, hipStream_t s);

size_t elastic_workspace_bytes(int n, int H, int W);
hipError_t launch_elastic_fields(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha,
                                 int radius, int32_t *off, void *ws, hipStream_t s);
void box_radii(double sigma, int r[3]);
size_t box_workspace_bytes(int n, int H, int W);
hipError_t launch_elastic_fields_box(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha,
                                     int32_t *off, void *ws, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s);
hipError_t launch_grid_tables(const double *grid, int n, int H, int W, int32_t *mapx, int32_t *mapy, hipStream_t s);
hipError_t launch_elastic_grid_u8(const uint8_t *img, const uint8_t *mask, int n, int H, int W, int C,
                                  const int32_t *off, const int32_t *mapx, const int32_t *mapy, uint8_t *out,
                                  uint8_t *out_mask, int per_image, hipStream_t s);
hipError_t launch_boxes_distort(const float *boxes, const int32_t *box_off, int n, int H, int W, const int32_t *off,
                                const int32_t *mapx, const int32_t *mapy, float *out, hipStream_t s);
hipError_t launch_ragged_masks(const miaug_ragged_args *a, int K, uint8_t *out, hipStream_t s);
size_t chain_f32_workspace_bytes(int n, int C, int H, int W);
hipError_t launch_chain_f32_fwd(const float *x, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                                const int32_t *mapy, float *y, void *ws, hipStream_t s);
hipError_t launch_chain_f32_bwd(const float *gy, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                                const int32_t *mapy, float *gx, void *ws, hipStream_t s);

hipError_t launch_image_stats(const uint8_t *img, int n, int64_t npix, int C, uint64_t *sum, int32_t *mn, int32_t *mx,
                              uint32_t *hist, hipStream_t s);

}  // namespace miaug
