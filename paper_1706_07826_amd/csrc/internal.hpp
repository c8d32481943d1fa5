// Internal declarations shared by the host half of libspvar (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "spvar.h"

namespace spv {

constexpr int kDigitBits = 9;
constexpr int kDigitSize = 512;
constexpr int kTopK = 10;
constexpr int kMaxColours = 16;
constexpr int kMaxDegree = 64;
constexpr int kMaxN = 65535;  // positions are packed into 16 bits

// A grow-only device allocation owned by the context.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// An instance together with the two bounds the library derives from its CSR at
// ingest (the samplers size their tables, digits and layouts by them).  Reduced
// problems keep their parent's bounds, which stay upper bounds: fixing only
// removes couplers, and |h'_u| + sum_{j free} |J_uj| <= |h_u| + sum_j |J_uj|.
struct Inst : spv_problem {
    int32_t max_degree = 1;  // longest row (1 when no row has an entry)
    int32_t x_bound = 0;     // max_i |h_i| + sum_j |J_ij|
    int32_t class_n[16] = {};  // variables per colour class when counted at ingest (all 0: unknown;
                               // reduced problems do not inherit them); launch planning only
};

// Ingest flags: also check the colour classes (every sampling call needs them);
// or the graph structure only (row_ptr and col; J, h and colour are not read).
constexpr int kIngestColours = 1;
constexpr int kIngestStructure = 2;

// Packed instance image written by the prep kernel (device memory):
//   int32 header[kImgHeader]: n, D, C, class_start[C+1] (padded to 32 entries)
//   int32 order[n]    position p -> original variable i (colour-major, index order)
//   int32 pos_of[n]   original variable i -> position p
//   int32 hpos[n]     bias of the variable at position p
//   uint32 nbr[n*D]   ELL neighbour records by position: (pos_j << 16) | (uint16)J_ij,
//                     padded with (p << 16) | 0 (self, zero coupling)
constexpr int kImgHeader = 32;

inline size_t image_words(int n, int D) { return (size_t)kImgHeader + 3ull * n + (size_t)n * D; }

struct TableCache {
    std::vector<double> betas;
    int scale = -1;
    int nd = -1;
    int row_len = -1;
    int unit = -1;
};

struct PtTableCache {
    std::vector<double> betas;
    int scale = -1, nd = -1, row_len = -1;
    void *dev = nullptr;  // the pt_tab allocation the blob was uploaded to
};

struct Ctx {
    int device = 0;
    int num_cus = 0;
    size_t lds_max = 0;
    std::string err;
    DevBuf image;
    DevBuf tables;
    DevBuf tables2;
    DevBuf scratch;
    DevBuf scratch2;
    DevBuf rounds;  // iterated-SPVAR working set
    DevBuf pt;      // parallel-tempering scratch: top-10 storage, boundary exchange
    DevBuf pt_tab;  // parallel-tempering tables (Metropolis rows, swap rows, swap digits)
    PtTableCache pt_cache;
    DevBuf batch;   // batched launch: descriptors, items, counter, images
    DevBuf top;     // sample assembly: per-list offsets
    DevBuf serve;   // serving slot: assembled tempering sample
    DevBuf merge;   // component count and recombination scratch
    DevBuf ms;      // multi-start working set
    void *ms_host = nullptr;  // pinned staging of the multi-start driver's per-start values
    size_t ms_host_bytes = 0;
    DevBuf tree;    // tree pre-processing scratch
    DevBuf sa_stream;  // streamed SA: task counter, tagged spin words between chunks
    DevBuf sa_big;     // SA: byte-parallel instance in global memory (problems too large for LDS)
    DevBuf sqa;        // SQA: inter-slice coupling per sweep
    DevBuf ingest;     // instance ingest: descriptors and results
    void *ingest_host = nullptr;  // pinned staging of the ingest descriptors and results
    size_t ingest_host_bytes = 0;
    TableCache tcache;
    std::vector<uint32_t> host_tables;
    void *batch_host = nullptr;  // pinned staging of descriptors and items
    size_t batch_host_bytes = 0;
    hipEvent_t batch_done = nullptr;
    hipStream_t capture_stream = nullptr;
    struct GraphEntry {
        std::vector<long long> key;
        hipGraphExec_t exec = nullptr;
        hipStream_t stream = nullptr;
    };
    std::vector<GraphEntry> graphs;
    struct TuneEntry {
        std::vector<long long> key;
        int threads, qw, wgs_per_cu;
        float ms;
        bool paired;
    };
    std::vector<TuneEntry> tuned;
    int last_shape[3] = {0, 0, 0};
    int last_sa_shape[5] = {0, 0, 0, 0, 0};  // spv_sample: threads, quads per workgroup, words per lane,
                                              // chunks, instance in global memory
    float last_tuned_ms = -1.f;
    // A context owned by one stream (serving slots) uploads tables
    // stream-ordered through pinned staging instead of draining the device.
    bool stream_private = false;
    hipStream_t own_stream = nullptr;
    void *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
};

// Host -> device copy of `bytes` into dst (grown as needed): stream-ordered
// through pinned staging for stream-private contexts, synchronous otherwise.
spv_status upload(Ctx *c, DevBuf &dst, size_t dst_off, const void *src, size_t bytes, hipStream_t s);

void batch_release(Ctx *c);

// ---- host helpers (api.cpp) ----
spv_status set_err(Ctx *c, spv_status st, const char *fmt, ...);
spv_status ensure(Ctx *c, DevBuf &b, size_t bytes);
spv_status hip_check(Ctx *c, hipError_t e, const char *what);
int digits_for(int64_t x_bound);
int table_row_len(int64_t x_bound);
uint32_t threshold_word(double beta, int64_t unit, int scale_log2, int digit, uint32_t d);
int swap_digits(double dbeta, int scale_log2);
spv_status check_problem_host(Ctx *c, const spv_problem *P);
// Validates B problems on the device (CSR shape and symmetry, coupler range, and
// with kIngestColours the colour classes) and derives each one's bounds into
// out[b]; waits for stream s.  The first failure sets the status and message.
spv_status ingest(Ctx *c, const spv_problem *P, int B, int flags, hipStream_t s, Inst *out);
spv_status check_betas(Ctx *c, const double *b, int count);
spv_status upload_tables(Ctx *c, DevBuf &dst, const double *betas, int count, int unit, int scale,
                         int nd, int row_len, hipStream_t s);

// The sampling entry points on an ingested instance (the public calls ingest
// first; internal drivers pass reduced problems that keep their parent's bounds).
spv_status sample_inst(spv_ctx *ctx, const Inst *P, const double *betas, int32_t sweeps, int32_t reads,
                       uint64_t seed, uint32_t sweep_offset, const int8_t *init_spins, int8_t *spins,
                       int64_t *energies, hipStream_t stream);
spv_status sqa_inst(spv_ctx *ctx, const Inst *P, const double *betas, const double *gammas, int32_t sweeps,
                    int32_t trotter, int32_t reads, uint64_t seed, int8_t *spins, int64_t *energies,
                    hipStream_t stream);
spv_status pt_inst(spv_ctx *ctx, const Inst *P, const spv_pt_params *prm, const spv_pt_out *out,
                   hipStream_t stream);
spv_status sample_batch_inst(spv_ctx *ctx, int32_t B, const Inst *problems, const double *betas, int32_t sweeps,
                             const int32_t *reads, const uint64_t *seeds, int8_t *const *spins,
                             int64_t *const *energies, const spv_batch_opts *opts, hipStream_t stream);

// Makes `dev` current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// ---- launchers (device translation units) ----
// Instance ingest (ingest.hip): one descriptor and one result per problem.
struct IngestDesc {
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const uint8_t *colour;
    int32_t n, nnz, n_colours;
    int32_t check_colours;  // 0: none, 1: range and independence, 2: range only (race-detection runs)
};
struct IngestResult {
    unsigned long long first_bad;  // (row + 1) << 8 | check of the first failure; ~0 when valid
    unsigned long long x_max;      // max_i |h_i| + sum_j |J_ij|
    int32_t max_degree;
    int32_t pad;
    long long pad2;
    int32_t class_n[16];           // variables per colour class (with the colour check)
};
enum IngestCheck : unsigned {
    kChkRowPtrEnds = 0,   // row_ptr[0] != 0 or row_ptr[n] != nnz (row 0: the whole problem)
    kChkRowPtrOrder = 1,  // row_ptr decreases, or leaves [0, nnz]
    kChkDegree = 2,       // more than kMaxDegree entries in a row
    kChkColourRange = 3,  // colour[i] >= n_colours
    kChkColRange = 4,     // col outside [0, n)
    kChkSelfLoop = 5,
    kChkUnsorted = 6,     // columns not strictly increasing
    kChkJRange = 7,       // |J| > 32767
    kChkColourEdge = 8,   // an edge inside a colour class
    kChkNoTranspose = 9,  // J(j, i) missing or different from J(i, j)
};
hipError_t launch_ingest(const IngestDesc *d, IngestResult *r, int B, int n_max, hipStream_t s);
// Packs the CSR into the position-ordered ELL image (one workgroup).
hipError_t launch_prep(const Inst *P, int32_t *image, hipStream_t s);

struct SaLaunch {
    const int32_t *image;
    int n, D, C;
    const uint32_t *tables;  // [sweeps][row_len]
    int row_len, nd;
    int sweeps;
    uint32_t sweep_offset;
    uint64_t seed;
    int reads;
    const int8_t *init;
    int8_t *out;
    int64_t *energies;
    int qw;       // quads (4 replicas) per workgroup
    int threads;  // workgroup size
    int wpl = 1;  // byte-parallel body: quad words per lane (2 needs qw = 2)
    int spin_limit = 1 << 22;  // streamed launch: bounded wait for a group's previous chunk
    bool global_instance = false;  // the instance stays in global memory (does not fit the LDS)
    unsigned char *big = nullptr;  // byte-parallel body with global_instance: its instance buffer
                                   // (sa_big_bytes); the general body reads the image itself
};
hipError_t launch_sa(const SaLaunch &L, hipStream_t s, size_t lds_limit);
// Simulated quantum annealing: one workgroup per read, P Trotter slices in LDS.
struct SqaLaunch {
    const int32_t *image;
    const uint32_t *tables;  // [sweeps][row_len] at beta_t / P
    const int32_t *jp;       // [sweeps]
    int8_t *out;
    int64_t *energies;
    int n, D, C, row_len, nd, sweeps, reads, P, threads, x_bound;
    bool global_instance = false;  // the instance stays in the global image
    uint64_t seed;
};
hipError_t launch_sqa(const SqaLaunch &L, hipStream_t s);
size_t sqa_lds_bytes(int n, int D, int row_len, int P, bool big = false);
// Streamed launch of the byte-parallel body (resident workgroups, chunked sweeps).
int sa_stream_plan(const SaLaunch &L, int num_cus, int force_grid);  // 1: use launch_sa
size_t sa_stream_bytes(int n, int reads, int qw);
hipError_t launch_sa_stream(const SaLaunch &L, int plan, void *buf, hipStream_t s);
int sa_stream_chunks_of(const SaLaunch &L, int plan);
size_t sa_lds_bytes(int n, int D, int row_len, int qw, bool big = false);
size_t sa_big_bytes(int n, int D);
bool sa_use_swar(int nd, int row_len);

hipError_t launch_energy(const int32_t *image, int n, int D, const int8_t *spins, int R,
                         int64_t *E, hipStream_t s);

struct FixLaunch {
    const spv_problem *P;
    const int32_t *image;
    const int8_t *samples;
    const int64_t *energies;
    int R, m, kmin, gauge_mode;  // gauge_mode: 0 off, 1 on, 2 auto
    const spv_fix_out *out;
    void *scratch;
    size_t scratch_bytes;
};
size_t fix_scratch_bytes(int n, int R, int m);
// Allocation-free persistence: the largest scratch it serves, and the per-device
// address of its file-scope scratch array (looked up once per device, with that
// device current).
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void **ptr);
hipError_t launch_compose(int n_cur, const uint8_t *fm_round, const int8_t *fv_round,
                          const int32_t *orig_cur, uint8_t *fixed_mask, int8_t *fixed_val,
                          const int64_t *info, const int32_t *orig_out, int32_t *orig_new,
                          hipStream_t s);
hipError_t launch_iota(int n, int32_t *a, uint8_t *fm, int8_t *fv, hipStream_t s);
hipError_t launch_persist_fix(const FixLaunch &L, hipStream_t s);
hipError_t launch_top_gather(const int8_t *ts, const int64_t *te, const int32_t *cnt, const int32_t *off,
                             int lists, int n, int8_t *S, int64_t *E, hipStream_t s);

// Device descriptor of one instance of a batched launch.
struct BatchInst {
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const uint8_t *colour;
    int8_t *out;
    int64_t *energies;
    uint64_t seed;
    long long image_off;  // int32 words into the image buffer
    int n, nnz, D, C, reads, pad;
};

struct BatchLaunch {
    const BatchInst *insts;
    const int32_t *items;  // [n_items][2]
    int n_items;
    int *counter;
    const int32_t *images;
    const uint32_t *tables;
    int row_len, nd, sweeps, qw, n_max, D_max, grid, threads;
    int dk;  // every image padded to this many records per site (0: per-instance degree)
    uint32_t sweep_offset;
    bool paired = false;  // paired body (items are instance, first quad, copies of 2 quads)
    int pairs_qw = 0;     // paired body: spin area of 2 n_max pairs_qw words
    int kmax = 0;         // paired body: most copies of an item
};
// Small instances get up to this many quads per work item (energy accumulators are sized for it).
constexpr int kBatchMaxItemQuads = 16;
size_t batch_lds_bytes(int n_max, int D_max, int row_len, int qw, int nd);
size_t batch_paired_lds_bytes(int n_max, int D_max, int row_len, int pairs_qw, int kmax);
hipError_t launch_batch_prep(const BatchInst *insts, int B, int n_max, int32_t *images, hipStream_t s);
hipError_t launch_batch_sa(const BatchLaunch &L, hipStream_t s);

// Race-detection build (SPV_LDS_SHADOW=1): the Metropolis class passes of the SA
// bodies check their LDS accesses against a bitmap that takes this much static LDS
// from every workgroup (so the planners' LDS limit is lowered by it).
#ifndef SPV_LDS_SHADOW
#define SPV_LDS_SHADOW 0
#endif
constexpr bool kLdsShadow = SPV_LDS_SHADOW != 0;
constexpr size_t kShadowLdsBytes = kLdsShadow ? 8192 : 0;
// Adds the counts of the unit's instrumented kernels to out[4] (write-write,
// read-write, passes checked, launches not covered); no-ops in the normal build.
hipError_t shadow_stats_sa(unsigned long long *out, bool reset);
hipError_t shadow_stats_batch(unsigned long long *out, bool reset);
hipError_t shadow_stats_pt(unsigned long long *out, bool reset);
hipError_t shadow_stats_ptx(unsigned long long *out, bool reset);
hipError_t shadow_stats_sqa(unsigned long long *out, bool reset);

// Checkpoint a tempering launch starts from (null members: fresh start).
struct PtResume {
    const int8_t *spins = nullptr;      // [runs][chains][K][n]
    const int8_t *top_spins = nullptr;  // [runs][Ls][10][n]
    const int64_t *top_E = nullptr;     // [runs][Ls][10]
    const int32_t *top_count = nullptr; // [runs][Ls]
};

struct PtLaunch {
    const int32_t *image;
    int n, D, C;
    int K, runs, chains, sweeps;
    uint32_t sweep_offset;
    uint64_t seed;
    int icm_lo, icm_hi, nw_icm;
    const uint32_t *mtab;  // [K][row_len]
    int row_len, nd;
    const uint32_t *stab;  // [K-1][7*512]
    const int32_t *snd;    // [K-1] swap digit counts (device)
    const spv_pt_out *out;
    void *scratch;         // top-10 states [runs][chains*(K/2)][10][n]
    int nqa;               // quads per run window
    int threads;
    PtResume resume;
};
size_t pt_lds_bytes(int n, int D, int K, int chains, int row_len, int nqa, int nw_icm);
hipError_t launch_pt(const PtLaunch &L, hipStream_t s);

// Tempering with each run's ladder split into G groups of m slots, one
// workgroup per (run, group); `big` reads the instance from the global image.
struct PtxLaunch {
    const int32_t *image;
    int n, D, C;
    int K, runs, chains, sweeps;
    uint32_t sweep_offset;
    uint64_t seed;
    int icm_lo, icm_hi, nw_icm;
    const uint32_t *mtab;
    int row_len, nd;
    const uint32_t *stab;
    const int32_t *snd;
    const spv_pt_out *out;
    int8_t *tops;             // [runs][Ls][10][n]
    uint32_t *xw;             // [runs][G][2][2][chains][ptx_msg_words(n)]
    int G, m, threads;
    bool big;
    bool esum;                // one slot pair per group: cluster energy terms gathered in the joins
    unsigned spin_limit;
    PtResume resume;
};
struct PtSplit {
    bool use = false, big = false, esum = false;
    int G = 1, m = 0, threads = 256, nw_icm = 0;
};
spv_status plan_pt_split(Ctx *c, int n, int D, int K, int runs, int chains, int row_len, int nd, int icm_lo,
                         int icm_hi, bool single_fits, PtSplit *sp);
unsigned pt_spin_limit();
// LDS claimed by one spv_pt_sample launch with the shapes it would pick.
spv_status pt_lds_footprint(Ctx *c, const Inst *P, int K, int runs, int chains, int icm_lo, int icm_hi,
                            int64_t *lds_total);
size_t ptx_lds_bytes(int n, int D, int m, int chains, int row_len, int nw_icm, bool big, bool esum);
int ptx_msg_words(int n);
hipError_t ptx_max_groups_resident(int nd, bool big, int D, int threads, size_t lds, int *blocks_per_cu);
hipError_t launch_ptx(const PtxLaunch &L, hipStream_t s);

// Components and sorted-merge recombination (components.hip).
size_t components_lds_bytes(int n);
hipError_t launch_components(const spv_problem *P, int32_t *comp, int32_t *count, hipStream_t s);
size_t merge_scratch_bytes(int C, int R);
hipError_t launch_merge(const spv_problem *P, const int32_t *comp, int C, const int8_t *S, int R, int8_t *merged,
                        int64_t *merged_E, int64_t *part_E, void *scratch, hipStream_t s);

// Multi-start driver helpers (multistart.hip).
// Per-start values of the current stage (device arrays in the driver's working set).
struct MsStageParams {
    const long long *off;  // [S] offset of the start's current problem (all reductions so far)
    const int *ncur;       // [S] variables of the start's current problem
    const int *n_prev;     // [S] the level's input size (0: the level did not run for the start)
    const int *n_next;     // [S] the level's output size
};
// Byte offsets of the fields of one reduction level slot (persistence or tree output).
struct MsLevelOffsets {
    size_t rp, col, J, h, co, orig, val, mask, kind, parent, round, order, info;
};
// The recorded energies of a start's sampling stages in stage order ([S][R[j]] each).
struct MsRecords {
    const long long *E[3];
    int R[3];
    int nst;
};
hipError_t launch_ms_record(int64_t *rec, int S, int R, const MsStageParams &prm, hipStream_t s);
hipError_t launch_ms_compose(const MsStageParams &prm, int S, int n, const unsigned char *lvl, size_t lvl_stride,
                             MsLevelOffsets lo, bool with_fixes, const int32_t *map_cur, int32_t *map_next,
                             uint8_t *fm, int8_t *fv, hipStream_t s);
hipError_t launch_ms_map_init(int32_t *map, int S, int n, int n_base, const int32_t *pre_orig, uint8_t *fm,
                              int8_t *fv, hipStream_t s);
hipError_t launch_ms_best(const MsRecords &rc, int S, int64_t *sb_E, int64_t *sb_pos, int64_t *best, hipStream_t s);
hipError_t launch_ms_lift(const int8_t *cur, int n_next, const int32_t *orig, const int8_t *val, int n_prev,
                          int8_t *prev, hipStream_t s);

// LDS read-bandwidth probe (probe.hip): synchronous on `s`; `out` receives at most
// 2 * num_cus words.
hipError_t run_lds_probe(int iters, int num_cus, uint32_t *out, double *bytes_per_s, hipStream_t s);
// Philox throughput probe (probe.hip): `out` receives at most 16 * num_cus words.
hipError_t run_philox_probe(int iters, int num_cus, uint32_t *out, double *blocks_per_s, hipStream_t s);

// Colour classes (colour.hip): prio [n] and info [4] are scratch.
size_t colour_lds_bytes(int n);
hipError_t launch_colour(const Inst *P, uint64_t seed, uint8_t *colour, uint32_t *prio, int *info,
                         hipStream_t s);

// Tree pre-processing (tree.hip).
size_t tree_scratch_bytes(int n);
bool tree_state_in_lds(int n, size_t lds_max);
hipError_t launch_tree_reduce(const spv_problem *P, const spv_tree_out *out, void *scratch, size_t lds_max,
                              hipStream_t s);
hipError_t launch_tree_complete(int n, const spv_tree_out *t, int n_free, int n_removed, const int8_t *reduced, int R,
                                int8_t *full, hipStream_t s);

}  // namespace spv

// The opaque context handle of the ABI.
struct spv_ctx {
    spv::Ctx c;
};
