// Internal declarations shared by the HIP translation units of libffs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "args.h"

namespace ffsk {

// ------------------------------------------------------------ Philox ------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// 4x32 S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key bumps
// 0x9E3779B9 / 0xBB67AE85.  Key = (seed lo, seed hi); counter =
// (sample lo, sample hi, step, stream).
struct Words {
  uint32_t w0, w1, w2, w3;
};

// Counter word 3 names the stream: 0 for the sampler's column order and
// uniforms, 1 for the eigenvector selection of the DPP front end.
__host__ __device__ inline Words philox_stream(uint64_t seed, uint64_t sample,
                                               uint32_t step, uint32_t stream) {
  uint32_t c0 = (uint32_t)sample, c1 = (uint32_t)(sample >> 32);
  uint32_t c2 = step, c3 = stream;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return Words{c0, c1, c2, c3};
}

__host__ __device__ inline Words philox_block(uint64_t seed, uint64_t sample,
                                              uint32_t step) {
  return philox_stream(seed, sample, step, 0u);
}

// Lazy Fisher-Yates: index in [t, n) from words 0,1 by 64-bit multiply-high.
__host__ __device__ inline int fy_index(Words w, int t, int n) {
  const uint64_t v = ((uint64_t)w.w1 << 32) | w.w0;
  const unsigned __int128 p = (unsigned __int128)v * (uint64_t)(n - t);
  return t + (int)(uint64_t)(p >> 64);
}

// 53-bit uniform in [0, 1) from words 2,3.
__host__ __device__ inline double uniform53(Words w) {
  const uint64_t v = ((uint64_t)w.w3 << 32) | w.w2;
  return (double)(v >> 11) * 0x1.0p-53;
}

// bfloat16 bits of x, rounded to nearest even (x finite).  Split-BF16
// plans carry Gamma as head = bf16(x) and tail = bf16(x - head).
__device__ inline uint32_t bf16_rn(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// ------------------------------------------------------- status bits ------
enum : int32_t { DEV_NUMERICAL = 1, DEV_BADCOLS = 2 };

// Tile sizes of the batched contraction.  Sites are padded to a multiple of
// SITE_PAD and samples to a multiple of SAMPLE_PAD so that every tile is
// full; padded sites carry zero rows of U (weight 0, never drawn) and padded
// samples zero columns of Gamma (results discarded).
constexpr int SITE_PAD = 256;  // multiple of the tile (128) and RCHUNK
constexpr int SAMPLE_PAD = 128;
constexpr int BLK = 32;        // sites per float64 partial sum
constexpr int RCHUNK = 64;     // sites per float64 chunk in the redraw product

// Device buffers of one batch of S samples (S_pad rows).
struct Work {
  int S_pad = 0;
  int32_t* perm = nullptr;     // [S_pad][N]   column order, in-place FY
  int32_t* xs = nullptr;       // [S_pad][N]   drawn sites
  void* F = nullptr;           // [S_pad][N][N] float64/complex128 factors
  void* beta = nullptr;        // [S_pad][N]   beta of the current step
  double* logdet = nullptr;    // [S_pad]
  void* gam = nullptr;         // [S_pad][Kg]  Gamma in bulk precision (split-BF16
                               // plans: per 16 k, 16 bfloat16 heads, 16 tails)
  uint32_t* occ = nullptr;     // [S_pad][L_pad/32] occupancy bitmap
  void* wh = nullptr;          // [S_pad][L_pad] bulk weights
  double* bsum = nullptr;      // [S_pad][L_pad/32] float64 block sums
  int32_t* ctl = nullptr;      // [0] flag count, [1] device status
  int32_t* flag_list = nullptr;// [S_pad]
  unsigned long long* counters = nullptr;  // [0] flagged [1] changed
  double* wr = nullptr;        // [S_pad][L_pad] float64 weights of flagged draws
  double* cs = nullptr;        // [S_pad][L_pad/RCHUNK] their chunk sums
  void* g64 = nullptr;         // [S_pad][Np] their dense float64 Gamma
  int32_t* forced = nullptr;   // [N] teacher-forced sites (test hook)
  int32_t* cmap_buf = nullptr; // [S_pad][N] room for per-sample column maps
  const int32_t* cmap = nullptr; // set (= cmap_buf) by column-subset calls
  const uint64_t* sid = nullptr; // [S] Philox sample indices (variable-size DPP runs)
  int32_t* fslot = nullptr;      // [S_pad] redraw slot of the current draw, -1 if none
  // deferred resolution: records of flagged draws (rec_cap = 0: not carved)
  // and the samples listed for a replay
  int rec_cap = 0;
  int32_t* rec_meta = nullptr;   // [rec_cap][4]
  void* rec_g = nullptr;         // [rec_cap][Np]
  uint32_t* rec_occ = nullptr;   // [rec_cap][L_pad/32]
  int32_t* rec_ctl = nullptr;    // [0] records taken, [1] samples listed
  int32_t* div = nullptr;        // [S_pad]
  int32_t* rep_row = nullptr;    // [S_pad]
  uint64_t* rep_sid = nullptr;   // [S_pad]
};

struct Dims {
  int L, N;       // sites, particles
  int ldu;        // columns of U (row stride of the float64 copy); = N unless
                  // a call samples column subsets of U
  int L_pad;      // sites padded to SITE_PAD
  int Np;         // N padded to 32 (contraction K chunk)
  int Kg;         // Gamma row length: Np (real) or 2*Np (complex)
  int cplx;       // complex128 input
  int bulk64;     // float64 bulk weights (plain path)
  int bf16;       // split-bfloat16 contraction (batched path)
};

// Raise a kernel's dynamic-LDS limit above the 64 KiB default when needed
// (gfx950 has 160 KiB of LDS per CU).
template <typename Kern>
inline void allow_lds(Kern kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

// Kernel launchers (defined in the .hip files).
void launch_init(const Dims& d, const Work& w, int S, hipStream_t st);
// Variable-size DPP runs (dpp.hip): x rows of width N set to -1 and logdet
// to 0; rows pos[i] of src (width lds) gathered into dst (width k); bucket
// results scattered back; device status and guard counters summed over the
// buckets (acc: [0] status bits, [1] flagged, [2] changed) and stored into
// the last bucket's slot for ffs_check.
void launch_fill_rows(int32_t* x, double* logdet, int n, int N, hipStream_t st);
void launch_gather_rows(const int32_t* src, int lds, const int32_t* pos, int n, int k,
                        int32_t* dst, hipStream_t st);
void launch_scatter_rows(const int32_t* xb, const double* ldb, const int32_t* pos, int n, int k,
                         int32_t* x, int ldx, double* logdet, hipStream_t st);
void launch_stats_add(const int32_t* ctl, const unsigned long long* counters,
                      unsigned long long* acc, hipStream_t st);
void launch_stats_store(const unsigned long long* acc, int32_t* ctl,
                        unsigned long long* counters, hipStream_t st);

// Metropolis conditional update of step t for S samples (k_mh.hip).
void launch_mh(const Dims& d, const Work& w, const void* u64, const int32_t* anchor, int S,
               int t, int m_cond, int radius, uint64_t seed, uint64_t first, hipStream_t st);

// Steps per block of the batched factor state; the factor launch after step
// t closes a block when t % kFactorBlock == kFactorBlock - 1.
constexpr int kFactorBlock = 16;
inline bool factor_closes_block(int t) { return t % kFactorBlock == kFactorBlock - 1; }

void launch_factor(const Dims& d, const Work& w, const void* u64, int S,
                   int t_upd, int t_solve, int n_steps, uint64_t seed,
                   uint64_t first_sample, hipStream_t st);
size_t factor_state_bytes(const Dims& d);  // per sample, batched path
// ev0 / ev1 (optional): events that the launch itself records around the
// dispatch; stamp (optional, device): receives the launch's span on the
// steady clock, [0] = min over the first workgroups' starts, [1] = max over
// all workgroups' ends (initialise to ULLONG_MAX, 0).
void launch_weights(const Dims& d, const Work& w, const void* ubulk_t,
                    const void* ubf, int S, hipStream_t st,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    unsigned long long* stamp = nullptr);
void launch_draw(const Dims& d, const Work& w, int S, int t, uint64_t seed,
                 uint64_t first_sample, double delta, double coef, int n_forced,
                 hipStream_t st);
void launch_repair(const Dims& d, const Work& w, const void* u64t, int S,
                   int t, uint64_t seed, uint64_t first_sample,
                   hipStream_t st);
// Deferred resolution: the fused per-step launch (draw of step t_upd, then
// the factor launch of launch_factor) and the end-of-call float64 check of
// the recorded draws (float64 product and redraw per chunk of S_pad
// records; samples whose site moves are listed for a replay).
void launch_drawfactor(const Dims& d, const Work& w, const void* u64, int S, int t_upd,
                       int t_solve, int n_steps, uint64_t seed, uint64_t first_sample,
                       double delta, double coef, int row0, hipStream_t st);
void launch_check_records(const Dims& d, const Work& w, const void* u64t, uint64_t seed,
                          uint64_t first_sample, int row0, hipStream_t st);
// Rows of a replay batch (xs, logdet of w) into the caller's output rows.
void launch_scatter_out(const Dims& d, const Work& w, int n, int n_keep, const int32_t* rows,
                        int32_t* x_out, double* logdet_out, hipStream_t st);
void launch_copy_out(const Dims& d, const Work& w, int S, int n_keep,
                     int32_t* x_out, double* logdet_out, hipStream_t st);
void launch_colmap(const Dims& d, const Work& w, const int32_t* cols, int S,
                   hipStream_t st);
void launch_plain(const Dims& d, const void* u64, const void* u64t,
                  const void* ubulk_t, uint64_t seed, uint64_t sample,
                  int n_keep, double delta, double coef, void* scratch, int32_t* x_out,
                  double* logdet_out, int32_t* ctl,
                  unsigned long long* counters, hipStream_t st);
size_t plain_scratch_bytes(const Dims& d);
void launch_density(const Dims& d, const void* ubulk_t, double* rho,
                    hipStream_t st);

// Tile variants of the float32 contraction (k_weights.hip) and the tuning
// table that picks one per launch shape (tune.hip).
struct TileShape {
  int sites, cols, kc, base;  // base: the variant of this tile with kc = 32
};
extern const TileShape kTiles[];
constexpr int kNumTilesDecl = 8;
bool tile_allowed(const Dims& d, int v);
void launch_weights_variant(const Dims& d, const WArgs& g, int s_round, int v,
                            hipStream_t st, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
int tile_choice(const Dims& d, int s_round);

// Argument blocks and grouped (multi-instance) launches.
WArgs make_wargs(const Dims& d, const Work& w, const void* ubulk_t);
DArgs make_dargs(const Dims& d, const Work& w, int S, uint64_t seed,
                 uint64_t first, double delta, double coef, int n_forced);
RArgs make_rargs(const Dims& d, const Work& w, const void* u64t, uint64_t seed,
                 uint64_t first);
FArgs make_fargs(const Dims& d, const Work& w, const void* u64, int n_steps,
                 uint64_t seed, uint64_t first);
int weights_group_items(const Dims& d, int S, int variant);
// The split-BF16 contraction (s_round samples, a multiple of the sample
// padding) of a plan's bfloat16 copy ubf of U; g as for the float32 one.
void launch_weights_bf16(const Dims& d, const WArgs& g, const void* ubf, int s_round,
                         hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
int weights_bf16_group_items(const Dims& d, int S);
void launch_weights_bf16_group(const GInst* inst, const GList& l, bool cplx, hipStream_t st);
int repair_group_items(const Dims& d, int S);
void launch_weights_group(const GInst* inst, const GList& l, bool cplx, int variant,
                          hipStream_t st);
void launch_draw_group(const GInst* inst, const GList& l, hipStream_t st);
void launch_repair_group(const GInst* inst, const GList& mma_l, bool cplx, hipStream_t st);
void launch_factor_group(const GInst* inst, const GList& l, bool cplx, int maxN,
                         hipStream_t st);
void launch_advance(GInst* inst, int n, hipStream_t st);

}  // namespace ffsk

// ---------------------------------------------- serving runtime hooks ------
// Implemented in api.hip, used by server.hip.
struct ffs_plan_s;
namespace ffsk {
size_t request_bytes(const ffs_plan_s* p, int64_t n, int* s_chunk);
int run_request(ffs_plan_s* p, void* base, int s_chunk, uint64_t seed,
                uint64_t first, int64_t n, int n_keep, int32_t* x, double* ld,
                hipStream_t st, unsigned long long* pinned);
const Dims& plan_dims(const ffs_plan_s* p);
int plan_device(const ffs_plan_s* p);
int plan_path(const ffs_plan_s* p);
int set_error(int st, const char* msg);
// For the grouped executor (group.hip).
struct PlanView {
  Dims d;
  const void *u64, *u64t, *ubulk, *ubf;
  double delta, coef;
  int64_t max_batch;
  int overlap;
};
PlanView plan_view(const ffs_plan_s* p);
size_t carve(const Dims& d, char* base, int S_pad, Work* w);
// Grouped executor pieces (group.hip), shared with the request server.
GInst make_ginst(const PlanView& pv, const Work& w, int S, int n_keep,
                 uint64_t seed, uint64_t first);
void start_instance(const PlanView& pv, const Work& w, int S, int n_keep,
                    uint64_t seed, uint64_t first, hipStream_t st);
// Work-item lists of a grouped tick: contraction per (tile variant, real)
// 0..3 and (variant 0/1, complex) 4..5, redraw product real/complex 6..7,
// factor real/complex 8..9 (which also finish the redraws), draw 10,
// split-BF16 contraction real/complex 11..12.
constexpr int kGroupLists = 13;
void group_items(const Dims& d, int S, int items[kGroupLists]);
void launch_tick(GInst* inst, const GList* gl, const int* maxN, int n_inst, hipStream_t st);

}  // namespace ffsk
