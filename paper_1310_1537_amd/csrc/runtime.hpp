// Host runtime shared by the entry points: context, data-set registry,
// per-stream scratch, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "glm.h"

namespace glmrt {

// ------------------------------------------------------------ errors

void set_error(const char* fmt, ...);
void clear_error();

#define GLM_FAIL(code, ...)            \
    do {                               \
        ::glmrt::set_error(__VA_ARGS__); \
        return (code);                 \
    } while (0)

#define GLM_HIP_CHECK(expr)                                                          \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            GLM_FAIL(GLM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

inline int elem_size(int dtype) {
    switch (dtype) {
    case GLM_F64: return 8;
    case GLM_F32: return 4;
    case GLM_BF16: return 2;
    case GLM_FP8_E4M3: return 1;
    }
    return 0;
}

// ------------------------------------------------------------ launch plan

// Which kernel instance and grid shape a data set is evaluated with.
struct Plan {
    int kind = 0;          // 0 = vector-chunk fused kernel, 1 = generic any-K kernel
    int lpr = 1;           // lanes per row
    int cpl = 1;           // 16-byte chunks per lane per row
    int rows_per_lane = 1; // R: row slots per lane per batch
    int wpb = 4;           // waves per block
    int nblocks = 1;
    int group = 32;        // blocks per merge group
    int interleave = 1;    // grid-strided batches (1) or contiguous ranges (0)
    const void* fn = nullptr;   // __global__ function
};

struct Dataset {
    glm_dataset_desc d;
    Plan plan;
};

// Column-major copy of a data set (differential update).
struct ColSet {
    glm_colset_desc d;
    std::vector<float> scale_host;   // FP8 column scales, read once at registration
};

// Device scratch of one stream: block partials, group partials, tickets.
struct Scratch {
    void* base = nullptr;
    size_t bytes = 0;
    double* partials = nullptr;
    double* gpart = nullptr;
    unsigned* counters = nullptr;
    size_t cap_partials = 0;   // doubles
    size_t cap_gpart = 0;      // doubles
    size_t cap_counters = 0;   // unsigned
};

// Device chain state of the on-device sampler for one stream: the proposal,
// f and g at the proposal, and the step counter.
struct SamplerBuf {
    double* buf = nullptr;
    size_t cap = 0;        // doubles
};

// Hessian buffers of one stream: row weights, block partials and the tile
// and block tables.
struct HessBuf {
    double* buf = nullptr;
    size_t cap = 0;            // doubles before the tables
    size_t ntick = 0;          // table capacity (ints)
    int* tiles = nullptr;      // per tile (row, column, first block, chunks), then per block (tile, chunk)
    int tiles_for = -1;        // tiles per side the tables were built for
    int64_t tiles_rows = -1;   // and the chunk cap ((N + 31) / 32) they used
};

struct GroupSet;   // defined by the batched entry point

}  // namespace glmrt

struct glm_ctx {
    int device = 0;
    int num_cu = 256;
    std::string arch;
    // options (glm_set_option)
    int blocks_per_cu = 1;
    bool interleave = true;
    bool matrix_cores = true;
    std::mutex mu;
    int64_t next_id = 1;
    std::unordered_map<int64_t, glmrt::Dataset> datasets;
    std::unordered_map<int64_t, glmrt::ColSet> colsets;
    std::map<void*, glmrt::Scratch> scratch;   // keyed by stream
    std::map<void*, glmrt::SamplerBuf> sampler;  // keyed by stream
    std::map<void*, glmrt::HessBuf> hess;        // keyed by stream
    hipStream_t own_stream = nullptr;
    // host-call staging (pinned) and device buffers
    double* h_stage = nullptr;
    double* d_stage = nullptr;
    size_t stage_cap = 0;   // doubles
};

namespace glmrt {

// Scratch for `stream` with room for the given sizes; grows (synchronising
// the device) when needed and zeroes the tickets of new memory.
glm_status get_scratch(glm_ctx* ctx, void* stream, size_t n_partials, size_t n_gpart,
                       size_t n_counters, Scratch** out);

// Sets the device of ctx current on this thread.
glm_status use_device(glm_ctx* ctx);

// Looks up (once per device; the device must be current) the device address
// of the allocation-free plain call's static scratch and clears its tickets.
glm_status static_scratch_setup(int device);

// Plan for a data set (defined with the kernel table).
glm_status make_plan(glm_ctx* ctx, const glm_dataset_desc& d, Plan* plan);

// Kernel instance evaluating up to nb coefficient vectors per pass over X
// for a plan's row geometry (nb is rounded down to an instantiated 1, 2, 4
// or 8 that fits the register budget); fn == nullptr if none.
struct MultiInst {
    const void* fn = nullptr;
    int R = 0;
    int NB = 0;
    const void* fleet = nullptr;   // the same geometry over several data sets per launch
    int wpb = 4;                   // waves per block of both forms
};
// The several-beta instance for nb_max vectors per pass; BF16 passes of three
// or more take the matrix-core form when mx is set and one exists.
MultiInst multi_instance(int dtype, int lpr, int cpl, int nb_max, bool mx);

// The matrix-core instance for BF16 rows of lpr lanes (4 vectors per pass),
// fn == nullptr where none is built.
MultiInst mx_instance(int lpr);

}  // namespace glmrt
namespace glmk {
struct FgParams;
struct FleetJob;
}
namespace glmrt {

// The kernel parameters launch_fused passes (partials, gpart and counters
// being the scratch regions of one evaluation).
void fused_params(const glm_dataset_desc& d, const Plan& pl, int NB, const double* betas,
                  const double* means, const double* precs, double prec, int nb, double* out,
                  double* partials, double* gpart, unsigned* counters, double* w_out,
                  const void* chain, glmk::FgParams* p);

// Launches a fleet instance (MultiInst::fleet) over nblocks blocks: jobs and
// blk_job (one job index per block) in device memory; every job's parameters
// are those launch_fused would pass for its data set, with blk0 its first
// block.
glm_status launch_fleet(const void* fn, int nblocks, int wpb, const glmk::FleetJob* jobs,
                        const uint16_t* blk_job, hipStream_t stream);

// Launches a fused kernel instance (NB slots) for nb coefficient vectors
// (betas nb x K, means nb x K or nullptr, precs nb or nullptr -> prec) into
// out (nb x (1 + K)); scratch must hold nblocks x NB x (1 + K) partials.
// w_out (NB == 1 only): per-row Hessian weights are written there when not
// nullptr.  chain (NB == 1 only): device address of a glmk::ChainParams; the
// launch then also takes one Metropolis step (its beta is the chain's
// proposal).
glm_status launch_fused(const glm_dataset_desc& d, const Plan& pl, const void* fn, int NB,
                        const double* betas, const double* means, const double* precs,
                        double prec, int nb, double* out, Scratch* s, hipStream_t stream,
                        double* w_out = nullptr, const void* chain = nullptr);

// Scratch sizes a plan needs for an NB-slot instance.
void scratch_need(const Plan& pl, int K, int NB, size_t* n_partials, size_t* n_gpart,
                  size_t* n_counters);

// Argument checks shared by every entry point that takes a data-set descriptor.
glm_status validate_desc(const glm_dataset_desc& d);

// Tuning cache: the launch choice found for a shape key, kept for the
// process and, when GLM_TUNE_CACHE names a file, persisted there as text
// lines "key a b us".
struct TuneEntry {
    int64_t a = 0;   // first tuned parameter (e.g. tile rows)
    int b = 0;       // second tuned parameter (e.g. blocks per compute unit)
    double us = 0;   // measured time of the choice
};
bool tune_cache_get(const std::string& key, TuneEntry* e);
void tune_cache_put(const std::string& key, const TuneEntry& e);

}  // namespace glmrt
