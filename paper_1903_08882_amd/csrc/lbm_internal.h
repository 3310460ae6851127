// lbm_internal.h -- shared between the kernels (kernels.hip) and the host API
// (api.hip) of the gfx950 thermal lattice Boltzmann library.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace lbmk {

constexpr int kQF = 19;            // D3Q19 populations
constexpr int kQG = 7;             // D3Q7 populations
constexpr int kNPop = kQF + kQG;   // planes in device memory
constexpr int kNPart = 24;         // doubles per block in the reduction scratch
constexpr int kRedBlock = 256;     // threads per block of the reduction kernels
constexpr uint32_t kFold = 256;    // blocks of the first reduction level
constexpr int kMaxN = 1600;        // keeps N^2 * N below 2^32 (index arithmetic)

// Relaxation and wall constants of one handle, in the arithmetic type R.
template <class R>
struct Coef {
    R s_a;      // 1/tau_f: energy, its square, the stresses (Sec. 2.2)
    R s_b;      // 8(2 tau_f - 1)/(8 tau_f - 1): energy fluxes, third-order moments
    R q_k, q_e, q_nu, a_T;   // D3Q7 rates and a_T (Sec. 2.3)
    R gbeta, T0;             // buoyancy g beta and reference temperature
    R abb_hot, abb_cold;     // (6 + a_T)/21 * T_w of the hot and cold walls
    R sf, isf;               // storage scale of f deviations and its inverse
    R sg, isg;               // storage scale of g and its inverse
    R drho_max;              // |rho - 1| above this marks a node as diverged
};

// Geometry of one launch: gx = ceil(N^2 / block) blocks per z-plane, gx * N
// blocks in all; block b of plane z covers in-plane indices r = b*block + t,
// with y = r / N.
struct Geo {
    int N;
    uint32_t N2;
    uint32_t gx;
    uint32_t magic;          // ceil(2^32 / N): y = umulhi(r, magic) for r < N^2
    uint32_t slab;           // storage bytes per z-plane (all 26 populations)
    uint32_t sub;            // storage bytes per sub-block
    uint32_t bbits, bmask;   // sub-block of 2^bbits nodes; bmask = 2^bbits - 1
};

// One cavity of a batch, as the batched step kernel sees it.
template <class R>
struct CavityDesc {
    Geo g;
    Coef<R> c;
    void *pop;         // the cavity's population storage
    int cell;          // LBM_SIDE_HEATED or LBM_RAYLEIGH_BENARD
    int active;        // 0: retired, its blocks do nothing
    uint32_t start;    // first logical block of the cavity in a batched launch
};

struct Layout {
    size_t esize = 0;        // bytes per stored moving population
    uint64_t node_bytes = 0; // storage bytes of one node's 26 populations
    uint32_t bbits = 0;      // log2 of the nodes per sub-block
    uint64_t sub = 0;        // storage bytes per sub-block
    uint64_t slab = 0;       // storage bytes per z-plane
    uint64_t pop_bytes = 0;  // storage bytes of all populations
    size_t off_pop = 0, off_macro = 0, off_snap = 0, off_wall = 0;
    size_t off_part = 0, off_fold = 0, off_res = 0, off_prof = 0, total = 0;
    uint32_t nblk_red = 0;   // blocks of the node-parallel reduction kernels
};

Layout make_layout(int N, int storage);

}  // namespace lbmk

struct lbm {
    lbm_params p{};
    lbm_opts o{};
    lbmk::Layout L{};
    lbmk::Geo geo{};
    int storage = 0;
    int block = 256;
    int waves[2] = {0, 0};   // occupancy cap of the step kernel (even, odd); 0 = none
    void *buf = nullptr;     // device buffer (caller's or ours)
    bool own_buf = false;
    int parity = 0;          // 0: planes hold f_i(x) in slot i; 1: post-collision swapped
    int64_t t = 0;           // steps since set_fields
    int64_t samples = 0;     // time-average samples taken
    bool initialised = false;
    bool has_flux = false;   // a step was taken since the populations were set
    bool pending_sample = false;   // the current state is a sample state whose
                                   // observables are not yet in the averages
    bool profiling = false;
    bool in_batch = false;   // stepped only through its batch
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    std::string err;
};

// A batch of cavities advanced together (each one an ordinary handle whose
// memory is a slice of the batch buffer).
struct lbm_batch {
    int K = 0;
    int storage = 0;
    int block = 256;
    int waves[2] = {0, 0};
    std::vector<lbm_t *> cav;
    std::vector<int> active;
    std::vector<double> last_res;      // last max |dT| of each cavity (inf before any check)
    void *buf = nullptr;
    bool own_buf = false;
    size_t off_table = 0;    // device copy of the descriptor table
    int parity = 0;
    int64_t t = 0;
    std::string err;
};

namespace lbmk {

// Launchers (kernels.hip).  All return the hipError_t of the launch.
hipError_t launch_init(const lbm_t *h, const double *uvwT, hipStream_t s);
hipError_t launch_set_pop(const lbm_t *h, const double *in, hipStream_t s);
hipError_t launch_get_pop(const lbm_t *h, double *out, hipStream_t s);
// One step; with obs, the step kernel also writes the observation planes
// [rho - 1, u, v, w, T] (arithmetic type) and wall fluxes of the state it
// starts from into the macro region (then launch_observe_reduce them).
hipError_t launch_step(const lbm_t *h, int parity, bool obs, hipStream_t s);
// FP64 planes [rho, u, v, w, T] of the current state.
hipError_t launch_macro(const lbm_t *h, double *macro_out, hipStream_t s);
// Observation planes and wall fluxes of the current state (outside a step).
hipError_t launch_obs_planes(const lbm_t *h, hipStream_t s);
// Reduces the observation planes (and wall fluxes) to the raw vector at
// res[0..]; with accumulate, also adds it to res[32..] and counts the sample.
hipError_t launch_observe_reduce(const lbm_t *h, bool accumulate, hipStream_t s);
// launch_obs_planes, then launch_observe_reduce.
hipError_t launch_observe(const lbm_t *h, bool accumulate, hipStream_t s);
hipError_t launch_reset_acc(const lbm_t *h, hipStream_t s);
// Residual against the snapshot into res[64..66], then snapshot := current.
hipError_t launch_residual(const lbm_t *h, hipStream_t s);
hipError_t launch_snapshot(const lbm_t *h, hipStream_t s);
// Batches: host image of the descriptor table (returns its size in bytes),
// total blocks of a batched launch, and the batched step.
hipError_t build_batch_table(const lbm_batch *b, void *host_table, size_t *bytes);
uint32_t batch_blocks(const lbm_batch *b);
hipError_t launch_step_batch(const lbm_batch *b, int parity, hipStream_t s);
// Fields (u, v, w, T) trilinearly resampled onto M^3 nodes, FP32 [4][M^3].
hipError_t launch_resample(const lbm_t *h, int M, float *out, hipStream_t s);
constexpr size_t kMaxDescBytes = 256;   // upper bound of sizeof(CavityDesc<double>)
// Dynamic LDS bytes that cap a block of `block` threads at `waves` waves per
// SIMD on the current device (0 when waves <= 0).
uint32_t lds_cap_bytes(int waves, int block);
// Library default occupancy caps (even, odd) of the step kernel per storage.
void default_waves(int storage, int out[2]);
// Centreline maxima of u (over z) and w (over x) into res[kResPeak..+3].
hipError_t launch_centerline(const lbm_t *h, hipStream_t s);
// Plane-averaged Nusselt profile across the cell: N values at
// off_prof + 2 N kProfG doubles (see lbm_nusselt_profile).
hipError_t launch_profile(const lbm_t *h, hipStream_t s);
// Streaming 16-byte copy of bytes (a multiple of 16) from src to dst.
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
constexpr int kProfGroups = 64;

// Offsets (in doubles) of the result block.
constexpr int kResCur = 0;
constexpr int kResAcc = 32;   // LBM_NRAW sums, then the sample count
constexpr int kResResid = 64;
constexpr int kResPeak = 72;
constexpr int kResDoubles = 96;

}  // namespace lbmk
