/*
 * spvar.h -- C ABI of the MI355X sample-persistence library (libspvar.so).
 *
 * The library implements the hot path of multi-start sample-persistence
 * variable reduction (SPVAR; Sec. II, Algorithms 1 and 2 of the paper):
 *   - the Monte Carlo samplers the method calls over and over: Metropolis
 *     simulated annealing and parallel tempering with isoenergetic
 *     (Houdayer) cluster moves (Sec. III.A, Sec. III.D.1), and
 *   - the persistence step: elite selection, per-variable agreement,
 *     fixing, and reduction of the Ising problem to (J', h', offset)
 *     (Algorithm 1; the zero-bias handling of Sec. II.C).
 *
 * Problem (Sec. I): minimise E(s) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i
 * over s in {-1,+1}^n, with integer couplers and biases; the real value of an
 * integer quantity q is q / 2^scale_log2.  Each undirected coupler is stored
 * twice in a symmetric CSR and counted once in E.
 *
 * Conventions
 *   - Pointers marked "device" are HIP device pointers on the context's
 *     device; "host" pointers are ordinary CPU memory.  Every output buffer
 *     is owned by the caller; the library never returns memory.  Scratch
 *     memory belongs to the context (allocated on first use, grown on
 *     demand, freed by spv_ctx_destroy).
 *   - Calls that take a stream enqueue work on it and return without waiting
 *     unless stated otherwise; host arguments are consumed before return.
 *   - Every function returns an spv_status; negative values are errors and a
 *     message is available from spv_last_error().  No exception crosses the
 *     ABI.  A context is not thread-safe: use one context per host thread.
 *   - Results depend only on the inputs and the seed, never on the stream,
 *     launch shape or batch composition (counter-based randomness).
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed & 0xffffffff, seed >> 32) and counters
 *   Metropolis digit j of (spin i, sweep t, replica r): (i, t, r>>2, 2<<24|j), word r&3
 *   initial spin i of replica r: (i, 0, r>>2, 1<<24), word r&3, +1 iff bit 31 set
 *   replica exchange (k,k+1) of chain-run c at sweep t, digit j: (k, t, c, 3<<24|j>>2), word j&3
 *   cluster move at slot k of run u at sweep t: (k, t, u, 4<<24), word 0
 *
 * Metropolis acceptance: x = -s_i f_i with f_i = h_i + sum_j J_ij s_j (the
 * flip changes E by 2x).  x <= 0 flips; otherwise, with x = sum_j d_j 512^j,
 * the flip is accepted iff every nonzero digit passes w_j < T_j[d_j],
 * T_j[d] = min(2^32-1, floor(2^32 exp(-(beta * (2 d 512^j)) / 2^scale_log2))),
 * tables built once per beta on the host in double precision.
 */
#ifndef SPVAR_H
#define SPVAR_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPV_OK = 0,
    SPV_EINVAL = -1,     /* malformed argument */
    SPV_EASYM = -2,      /* CSR is not symmetric / sorted / loop-free */
    SPV_ECOLOUR = -3,    /* an edge joins two variables of one colour class */
    SPV_ERANGE = -4,     /* a value exceeds a representable range */
    SPV_ECAPACITY = -5,  /* instance or batch does not fit the device layout */
    SPV_EBUDGET = -6,    /* request exceeds the serving budget */
    SPV_EDEVICE = -7,    /* HIP runtime error */
    SPV_EAGAIN = -8,     /* try again (queue full / result pending) */
    SPV_ENOMEM = -9,     /* allocation failed */
    SPV_EINTERNAL = -10  /* internal consistency check failed */
} spv_status;

typedef struct spv_ctx spv_ctx;

/*
 * An Ising instance (Sec. I) resident in device memory.
 *   n, nnz          host: variables and stored CSR entries (2 x couplers)
 *   row_ptr [n+1]   device: row_ptr[0] = 0, row_ptr[n] = nnz
 *   col [nnz]       device: strictly increasing per row, no self loops
 *   J [nnz]         device: int32, symmetric (J(i,j) == J(j,i)), |J| <= 32767
 *   h [n]           device: int32 biases
 *   colour [n]      device: colour class of each variable; no edge joins
 *                   two variables of one class (sweeps go class by class)
 *   n_colours       host: 1..16
 *   scale_log2      host: 0..30, real value = integer / 2^scale_log2
 * Every sampling call (spv_sample, spv_sqa_sample, spv_pt_sample,
 * spv_sample_batch, spv_ispvar, spv_multistart, spv_energy, and the server at
 * submission) ingests the instance first: one device pass validates the CSR
 * (row_ptr order and ends, columns in range, sorted, no self loops, equal
 * transposed entries, |J| <= 32767, at most 64 entries per row) and the colour
 * classes, and derives the two bounds the sampler is sized by, the longest row
 * and x_bound = max_i (|h_i| + sum_j |J_ij|), which must stay below 2^26.  The
 * call waits for `stream` to read them back; a failure returns its status
 * (SPV_EASYM, SPV_ECOLOUR, SPV_ERANGE, SPV_ECAPACITY) before any launch.
 * The arrays must not change while a call that reads them is in flight.
 */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const uint8_t *colour;
    int32_t n_colours;
    int32_t scale_log2;
} spv_problem;

/* Context on HIP device `device`.  *out receives the handle. */
spv_status spv_ctx_create(int32_t device, spv_ctx **out);
void spv_ctx_destroy(spv_ctx *ctx);
/* Message of the last failing call on this context ("" if none). */
const char *spv_last_error(const spv_ctx *ctx);
/* Library version string. */
const char *spv_version(void);

/*
 * Race detection (debug build of the library with SPV_LDS_SHADOW=1,
 * libspvar_shadow.so).  The Metropolis class passes of the SA, tempering and
 * SQA kernels (Sec. III.A, III.D.1; one colour class at a time) check, on every pass, that no spin
 * word is written by two tasks and that no task reads a neighbour word another
 * task of the pass writes, against a per-workgroup bitmap in LDS (8 KiB of LDS
 * per workgroup, taken from the planners' limit).  Conflicts are counted, never
 * trapped.  Waits for the device, then writes counts[0..3]: write-write
 * conflicts, read-write conflicts, class passes checked, launches whose spin
 * area exceeded the bitmap (unchecked); reset != 0 clears them.  SPV_EINVAL in
 * the normal build.  In the debug build only, the environment variable
 * SPVAR_SHADOW_ALLOW_COLOUR_EDGES lets colourings with an edge inside a class
 * through ingest (instead of SPV_ECOLOUR), so the detector can be shown the
 * races such a colouring causes; samples are then not reproducible.
 */
spv_status spv_debug_lds_shadow(spv_ctx *ctx, uint64_t counts[4], int32_t reset);

/*
 * Instance ingest on its own (Sec. I: the Ising instance J, h), synchronous
 * (waits for the device first): the validation every sampling call performs,
 * returning SPV_OK or the first violation.  On success the derived bounds are
 * written to max_degree (longest row, >= 1) and x_bound (max_i |h_i| +
 * sum_j |J_ij|); either pointer may be NULL.
 */
spv_status spv_problem_check(spv_ctx *ctx, const spv_problem *P, int32_t *max_degree, int32_t *x_bound);

/*
 * Simulated annealing (Sec. III.A sampler; one Metropolis sweep per beta).
 *   betas [sweeps]   host: inverse temperatures, >= 0 and finite
 *   reads            independent replicas r = 0..reads-1
 *   seed             Philox key
 *   sweep_offset     global index of the first sweep (resume support)
 *   init_spins       device [reads][n] int8 +-1 initial states, or NULL for
 *                    the Philox initial state
 *   spins            device [reads][n] int8: final state of each read
 *   energies         device [reads] int64: E of each final state
 * The sample is the final state of every read (not the best seen).
 * When the replicas need more workgroups than stay resident on the device, the
 * launch is streamed: resident workgroups take (replica group, chunk of sweeps)
 * tasks in order and carry each group's spins between chunks through context
 * scratch; the sample is bit-identical to the one-launch schedule.  A streamed
 * task waits (bounded) for its group's previous chunk; should a wait ever be
 * abandoned, every read of that group reports energy INT64_MIN.
 * An instance too large for the LDS beside its replicas' spins is read from
 * global memory (the LDS keeps the spins and threshold tables), so n is bounded
 * by the spins of one replica quad: 4n bytes plus the tables within the LDS
 * (about 37,000 variables; about 19,900 for the byte-parallel body, which holds
 * a complement plane).  SPV_ECAPACITY beyond that.
 */
spv_status spv_sample(spv_ctx *ctx, const spv_problem *P, const double *betas, int32_t sweeps,
                      int32_t reads, uint64_t seed, uint32_t sweep_offset,
                      const int8_t *init_spins, int8_t *spins, int64_t *energies,
                      hipStream_t stream);

/* Colour classes for the parallel sweep (the colour field of spv_problem):
 * independent sets that one Metropolis pass updates at once.  Jones-Plassmann
 * rounds: vertex v has priority (word 0 of Philox(v, 0, 0, 5 << 24) under `seed`,
 * then v), higher first; each round every uncoloured vertex that outranks all its
 * uncoloured neighbours (every CSR entry counts as an edge) takes the smallest
 * colour its coloured neighbours lack.  The result equals first-fit greedy in
 * decreasing priority order (at most max_degree + 1 colours).  P->colour and
 * P->n_colours are ignored.  colour: device [n] uint8 output; *n_colours (host)
 * receives the count; synchronous on `stream`.  ERANGE when more than 16 colours
 * would be needed (colour then holds a capped, invalid colouring); ECAPACITY when
 * 2n bytes exceed the LDS. */
spv_status spv_colour(spv_ctx *ctx, const spv_problem *P, uint64_t seed, uint8_t *colour, int32_t *n_colours,
                      hipStream_t stream);

/* Device LDS read bandwidth in bytes/s, measured by a probe kernel (two
 * 1024-thread workgroups per CU reading bank-conflict-free 16-byte words; one
 * timed launch of `iters` x 4 reads per lane after one warm-up launch).  The
 * measured denominator of the LDS rooflines of the sweeps.  Synchronous on
 * `stream`; uses context scratch.  EINVAL for iters outside [1, 2^24]. */
spv_status spv_lds_probe(spv_ctx *ctx, int32_t iters, double *bytes_per_s, hipStream_t stream);

/* Philox4x32-10 blocks per second of the device at full occupancy (16 waves per
 * CU, each lane chaining `iters` blocks; one timed launch after a warm-up).  The
 * VALU issue slots one block costs are (CUs x 64 lanes x clock) / this rate: the
 * measured basis of the sampler's VALU roofline.  Synchronous on `stream`; uses
 * context scratch.  EINVAL for iters outside [1, 2^24]. */
spv_status spv_philox_probe(spv_ctx *ctx, int32_t iters, double *blocks_per_s, hipStream_t stream);

/*
 * Simulated quantum annealing (Sec. III sampler "SQA": discrete-time
 * path-integral Monte Carlo of the transverse-field Ising model; the paper
 * names it without its parameters, so the Trotter number and both schedules
 * are the caller's).
 *   betas [sweeps]   host: inverse temperatures beta_t > 0, finite
 *   gammas [sweeps]  host: transverse fields Gamma_t > 0, finite (same units as
 *                    the couplings' real values)
 *   trotter          slices P per read: a multiple of 8 in [8, 256]
 *   reads            independent reads u = 0..reads-1
 *   seed             Philox key
 *   spins            device [reads][n] int8: each read's lowest-energy slice
 *                    after the last sweep (ties: lowest slice index)
 *   energies         device [reads] int64: E of that slice
 * Each sweep samples E_eff = sum_k E(s^k) - Jp_t sum_k sum_i s^k_i s^{k+1}_i
 * (slice ring) at inverse temperature beta_t / P, with Jp_t = round(P Jperp
 * 2^scale_log2) half away from zero and Jperp = -ln(tanh(beta_t Gamma_t / P)) /
 * (2 beta_t); sweeps visit the colour classes in order and, within a class,
 * the even slices, then the odd ones.  Slice k of read u uses replica index
 * u P + (k mod 2) P/2 + floor(k/2) for its Philox counters (Metropolis tag 6,
 * initial state tag 1).  Bit-identical to the oracle.  EINVAL for bad
 * arguments; ERANGE when Jp_t reaches 2^24 or x_bound + 2 max Jp needs more
 * than 3 base-512 digits; ECAPACITY when one read's P slices (P/4 words per
 * variable) and the two acceptance rows exceed a workgroup's LDS (the instance
 * itself is read from global memory when it does not fit beside them).
 */
spv_status spv_sqa_sample(spv_ctx *ctx, const spv_problem *P, const double *betas, const double *gammas,
                          int32_t sweeps, int32_t trotter, int32_t reads, uint64_t seed, int8_t *spins,
                          int64_t *energies, hipStream_t stream);

/* The launch shape the last spv_sample call on this context used: threads per
 * workgroup, quads (4 replicas) per workgroup, quad words per lane, sweep chunks
 * per group (1: one launch over all workgroups; more: streamed), and whether the
 * instance was read from global memory (1) rather than LDS (0). */
spv_status spv_sample_last_shape(const spv_ctx *ctx, int32_t *threads, int32_t *quads_per_wg,
                                 int32_t *words_per_lane, int32_t *chunks, int32_t *global_instance);

/* E(s) of R states: spins device [R][n] int8 +-1 -> energies device [R] int64. */
spv_status spv_energy(spv_ctx *ctx, const spv_problem *P, const int8_t *spins, int32_t R,
                      int64_t *energies, hipStream_t stream);

/*
 * Outputs of the persistence step.  All device pointers; the reduced CSR
 * buffers must hold P->n rows / P->nnz entries (outputs never exceed them).
 *   fixed_mask [n]  1 where the variable was fixed
 *   fixed_val  [n]  its value (+-1), 0 where free
 *   row_ptr [n+1], col [nnz], J [nnz], h [n], colour [n]: reduced problem
 *                   over the free variables, renumbered in index order
 *   orig_index [n]  reduced variable u -> original variable
 *   info [8]        int64: n_free, nnz_free, offset, n_fixed, pivot (-1 when
 *                   the gauge was not applied), m, k_min, status (0, or a
 *                   negative spv_status detected on the device: SPV_EINVAL
 *                   for an entry other than +-1 in an elite row (the only
 *                   rows read) or for an energy of INT64_MIN (the mark of an
 *                   abandoned streamed sample, spv_sample), SPV_ERANGE for an h' outside int32,
 *                   SPV_EINTERNAL for an unresolved gauge hash)
 */
typedef struct {
    uint8_t *fixed_mask;
    int8_t *fixed_val;
    int32_t *row_ptr;
    int32_t *col;
    int32_t *J;
    int32_t *h;
    uint8_t *colour;
    int32_t *orig_index;
    int64_t *info;
} spv_fix_out;

/*
 * Persistence and reduction (Algorithm 1: "Narrow down solutions to
 * elite_threshold percentile", "Find mean value of each variable",
 * "Fix variables ...", "Update J and h").
 *   samples [R][n]  device int8 +-1, energies [R] device int64
 *   elite_frac      (0, 1]: m = max(1, ceil(elite_frac * R)) rows with the
 *                   lowest (E, row index)
 *   threshold       (0, 1]: fix i iff |sum_elite s_ri| >= ceil(threshold*m),
 *                   to its sign
 *   gauge           0 off, 1 on, 2 on iff every h_i == 0 (zero-bias
 *                   handling, Sec. II.C): variables whose elite columns are
 *                   equal up to a global sign form classes; the pivot is the
 *                   lowest index of the largest class (ties: lower minimum
 *                   index); every elite row is multiplied by its pivot value
 *                   before counting, so the pivot's class is fixed.
 * Reduction: h'_u = h_u + sum_{j fixed} J_uj v_j, offset = sum_{i<j fixed}
 * J_ij v_i v_j + sum_{i fixed} h_i v_i, so E(s) = E'(s_U) + offset.
 * Asynchronous: info becomes valid when the stream reaches this point.
 */
spv_status spv_persist_fix(spv_ctx *ctx, const spv_problem *P, const int8_t *samples,
                           const int64_t *energies, int32_t R, double elite_frac,
                           double threshold, int32_t gauge, const spv_fix_out *out,
                           hipStream_t stream);

/*
 * spv_persist_fix for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and outputs, with its scratch in a file-scope device
 * array of 16 MiB per device (held until the process ends; its address is
 * looked up when a context is created on the device) instead of context
 * memory.  Calls no allocating routine and no memset.  SPV_ECAPACITY when the
 * call needs more scratch than that (about 64 + 4R + 8n ceil(m/64) + 8n +
 * 16 (power of two >= 2n) + 8n bytes, m the elite size).  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * different streams, or from different threads) race; calls ordered on one
 * stream do not.  The array keeps the last call's contents; each call writes
 * what it reads before reading it.
 */
spv_status spv_persist_fix_noalloc(spv_ctx *ctx, const spv_problem *P, const int8_t *samples,
                                   const int64_t *energies, int32_t R, double elite_frac,
                                   double threshold, int32_t gauge, const spv_fix_out *out,
                                   hipStream_t stream);

/*
 * Iterated SPVAR (Sec. II.B "ISPVAR"): `rounds` rounds of spv_sample
 * (round r uses seed + r) followed by spv_persist_fix on the current reduced
 * problem; fixes are never undone; stops early when nothing is left.
 * Synchronous (the host needs each round's reduced size).
 *   fixed_mask, fixed_val  device [n]: cumulative fixes, original indices
 *   round_info             host [rounds][4] int64: n_free after the round,
 *                          cumulative offset, best full-problem energy of the
 *                          round's sample (E' + offsets so far), variables
 *                          fixed in the round
 *   rounds_run             host: number of rounds executed
 */
spv_status spv_ispvar(spv_ctx *ctx, const spv_problem *P, const double *betas, int32_t sweeps,
                      int32_t reads, uint64_t seed, int32_t rounds, double elite_frac,
                      double threshold, int32_t gauge, uint8_t *fixed_mask, int8_t *fixed_val,
                      int64_t *round_info, int32_t *rounds_run, hipStream_t stream);

/*
 * Parallel tempering (Sec. III.D.1 "PTICM").  Each run holds `chains`
 * ladders of K slots (betas ascending).  One sweep = Metropolis on every
 * slot; replica exchange of pairs (k,k+1) with k = t (mod 2) in each chain
 * (D = E_k - E_{k+1}; D <= 0 swaps, else the digit test of D with tables of
 * dbeta = beta_{k+1} - beta_k); Houdayer cluster moves between chains 0 and
 * 1 at slots icm_lo..icm_hi-1 (chains == 2); then the K/2 coldest slots
 * (k >= K - K/2) are offered to per-slot lists of the 10 lowest-energy distinct
 * states seen (Sec. III.D.1 sample formation).
 * Replica index r = (run * chains + chain) * K + slot (keyed by slot, so the
 * random stream follows the temperature).
 * When K % 4 == 0 a run's ladder may be split over several workgroups of
 * consecutive slots (a multiple of 4 slots each, or with cluster moves on 2 or
 * 1) that decide the slot pairs straddling their boundaries from energies and
 * edge states published through global memory (the split is chosen from the
 * run count and the LDS footprint; results do not depend on it).  The
 * split launch is only made when all its workgroups fit on the device at
 * once; should a workgroup still wait for a neighbour beyond a bounded spin,
 * it stops and writes top_count = -1 for its lists (and spv_top_sample then
 * reports SPV_EINVAL).  SPV_ECAPACITY when no layout fits.
 *
 * Checkpoint and resume: the outputs of a call (final_spins and the three
 * top-10 arrays) are its checkpoint.  A call given them as resume_* with the
 * same problem, betas, runs, chains, seed and cluster-move slots, and with
 * sweep_offset advanced by the earlier call's sweeps, continues those runs:
 * N sweeps then a resumed M sweeps give the bits of one (N + M)-sweep call.
 *   resume_spins      device [runs][chains][K][n] int8 or NULL (Philox initial
 *                     state): the slots' starting states; a byte > 0 is +1,
 *                     any other byte -1; energies are recomputed from them
 *   resume_top_spins  device [runs][chains][K/2][10][n] int8, resume_top_E
 *                     [..][10] int64, resume_top_count [runs][chains][K/2]
 *                     int32: all three or all NULL (empty lists; with n = 0
 *                     resume_top_spins may be NULL alone).  Entries
 *                     0..count-1 of a list start it, as inserted before any
 *                     offer of this call in their listed order (spins read as
 *                     above; E taken as given, so pass the checkpoint's own
 *                     energies).  A count outside 0..10 (such as the -1 of an
 *                     abandoned wait) starts that list empty and its output
 *                     count is -1 again.
 * The resume arrays may be the very arrays `out` names (a run continued in
 * place); any other overlap with the outputs is undefined.  The serving loop's
 * tempering requests always start fresh.
 */
typedef struct {
    int32_t K;
    int32_t runs;
    int32_t chains;
    int32_t sweeps;
    const double *betas; /* host [K], ascending */
    uint64_t seed;
    uint32_t sweep_offset;
    int32_t icm_lo;
    int32_t icm_hi;
    const int8_t *resume_spins;
    const int8_t *resume_top_spins;
    const int64_t *resume_top_E;
    const int32_t *resume_top_count;
} spv_pt_params;

/* Any member may be NULL when not wanted.  All device pointers.
 *   final_spins [runs][chains][K][n], final_E [runs][chains][K]
 *   top_spins [runs][chains][K/2][10][n], top_E [..][10] (unfilled entries:
 *   E = INT64_MAX, spins 0), top_count [runs][chains][K/2]
 *   Entries of a list are ordered by (E, insertion). */
typedef struct {
    int8_t *final_spins;
    int64_t *final_E;
    int8_t *top_spins;
    int64_t *top_E;
    int32_t *top_count;
} spv_pt_out;

spv_status spv_pt_sample(spv_ctx *ctx, const spv_problem *P, const spv_pt_params *params,
                         const spv_pt_out *out, hipStream_t stream);

/*
 * Sample formation of a tempering run (Sec. III.D.1): the filled entries of
 * `lists` top-10 lists, concatenated in list order ([runs][chains][K/2] for
 * the output of spv_pt_sample), each list in its (E, insertion) order.
 *   top_spins [lists][10][n], top_E [lists][10], top_count [lists]: device
 *   spins [lists*10][n], energies [lists*10]: device, caller-owned (worst case)
 *   rows   host: number of rows written
 * Reads the counts back, so the call returns after the gather is queued and
 * `stream` has finished the work before it.  SPV_EINVAL for a count outside
 * 0..10.
 */
spv_status spv_top_sample(spv_ctx *ctx, const int8_t *top_spins, const int64_t *top_E,
                          const int32_t *top_count, int32_t lists, int32_t n, int8_t *spins,
                          int64_t *energies, int32_t *rows, hipStream_t stream);

/*
 * Connected components of a problem (Sec. II.C, special considerations: a
 * problem left disconnected by fixing is treated per component).  Edges are
 * the couplers with J != 0; components are numbered 0..n_comp-1 in order of
 * their smallest variable index.
 *   comp [n]  device int32, output
 *   n_comp    host, output; the call waits for `stream` to read it back
 */
spv_status spv_components(spv_ctx *ctx, const spv_problem *P, int32_t *comp, int32_t *n_comp,
                          hipStream_t stream);

/*
 * Sorted-merge recombination of a sample over the components (Sec. II.C): the
 * partial energy E_c(r) of component c in row r sums its couplers (each once)
 * and biases, so E = sum_c E_c; the rows of each component are ordered by
 * (E_c, row index); merged row k takes every component's variables from the
 * k-th row of that component's order, and merged_E[k] is the sum of those
 * partial energies.  The best merged row holds every component's best
 * partial solution, so it is a ground state whenever each component was
 * solved in at least one row.
 *   comp [n], n_comp   from spv_components (1 <= n_comp <= n)
 *   samples [R][n] int8, merged [R][n] int8 (must not overlap samples),
 *   merged_E [R] int64: device
 *   part_E [n_comp][R] int64: device, each component's partial energies in its
 *                      order, or NULL
 */
spv_status spv_merge_components(spv_ctx *ctx, const spv_problem *P, const int32_t *comp, int32_t n_comp,
                                const int8_t *samples, int32_t R, int8_t *merged, int64_t *merged_E,
                                int64_t *part_E, hipStream_t stream);

/*
 * Multi-start SPVAR (Algorithm 2), with the zero-bias handling of Sec. II.C and
 * the sample split of the parameter appendix.  [Optional] (preprocess bit 0)
 * the problem is tree pre-processed first (spv_tree_reduce).  Each of the
 * `starts` independent starts then runs these stages on its own current
 * problem; a sampling stage draws a sample of that problem and records its
 * energies in full-problem units (E' plus the offsets of every reduction so
 * far), and each reduction modifies the start's problem:
 *   correlation step (corr_reads > 0; before the SPVAR step when corr_after is
 *     0 -- the appendix's "pre-fixing" -- or after the SPVAR and tree steps
 *     when it is 1, the order the algorithm box lists): a sample of
 *     corr_reads, then spv_persist_fix with the gauge on, corr_elite_frac and
 *     corr_threshold, which fixes the pivot's class of perfectly
 *     (anti)correlated variables (threshold 1.0);
 *   SPVAR step (Algorithm 1): a sample of fixing_reads, then spv_persist_fix
 *     with gauge, elite_frac and threshold;
 *   [optional] (preprocess bit 1) tree pre-processing of the modified problem;
 *   solving step (solving_reads > 0): a sample of the modified problem,
 *     optionally recombined over its components (Sec. II.C).
 * The first sampling stage samples the problem all starts share: one job with
 * `seed`, start s owning reads [s*R, (s+1)*R).  The k-th later sampling stage
 * (k = 1, 2) of start s uses seed + 1 + (k-1)*starts + s (SA: one batched
 * launch over the starts; SQA, spv_sqa_sample: a launch per start).  A start
 * whose problem became empty records its offset.  The call waits for `stream`
 * (it reads back the per-start sizes after each reduction).
 */
typedef struct {
    int32_t starts;          /* num_starts, 1..4096 */
    int32_t corr_reads;      /* correlation step sample per start (0: no correlation step) */
    int32_t fixing_reads;    /* fixing_sample_size >= 1 */
    int32_t solving_reads;   /* solving_sample_size >= 0 */
    const double *betas;     /* host [sweeps]: the schedule of every sample */
    int32_t sweeps;
    uint64_t seed;
    double elite_frac;       /* SPVAR step, as spv_persist_fix */
    double threshold;
    int32_t gauge;
    double corr_elite_frac;  /* correlation step: correlation_elite_threshold, (0, 1] */
    double corr_threshold;   /* correlation_threshold, (0, 1] (1.0 in the paper) */
    int32_t corr_after;      /* 0: correlation step before the SPVAR step; 1: after it */
    int32_t preprocess;      /* bit 0: tree step before the loop; bit 1: after each SPVAR step */
    int32_t merge;           /* 1: recombine each solving sample over its components */
    int32_t sampler;         /* 0: SA; 1: SQA with `trotter` slices and the Gamma schedule `gammas` */
    int32_t trotter;         /* SQA: as spv_sqa_sample */
    const double *gammas;    /* SQA: host [sweeps] */
} spv_multistart_params;

typedef struct {
    int64_t *corr_E;         /* device [starts][corr_reads] (NULL when corr_reads == 0) */
    int64_t *fixing_E;       /* device [starts][fixing_reads] */
    int64_t *solving_E;      /* device [starts][solving_reads]: sorted when recombined */
    uint8_t *fixed_mask;     /* device [starts][n] or NULL: fixed by the correlation and SPVAR steps */
    int8_t *fixed_val;       /* device [starts][n] or NULL: their values (0 where not fixed) */
    int64_t *info;           /* host [starts][8] or NULL: fixed by the correlation step, fixed by
                                the SPVAR step, removed by the tree step, n_free of the final
                                problem, its offset, its components (0 unless recombined), the
                                correlation pivot (original index, -1 when none), 0 */
    int64_t *info_pre;       /* host [8] or NULL: spv_tree_reduce info of the pre-processing
                                (n, nnz, 0, ... when not applied) */
    int64_t *start_best;     /* host [starts] or NULL: each start's lowest recorded energy */
    int8_t *best_spins;      /* device [n] or NULL: the first lowest recorded state in the order
                                start 0 stage by stage, start 1, ..., lifted to the full problem
                                through the start's reductions in reverse */
    int64_t *best_E;         /* host or NULL */
} spv_multistart_out;

spv_status spv_multistart(spv_ctx *ctx, const spv_problem *P, const spv_multistart_params *params,
                          const spv_multistart_out *out, hipStream_t stream);

/* Per-start sample split of the parameter appendix for a total of `total`
 * reads: zero-bias problems give floor(2 total / 5) to the correlation step and
 * halve the rest between fixing (the odd read) and solving; otherwise fixing
 * and solving halve the total.  Any output pointer may be NULL.  Host only. */
void spv_multistart_split(int32_t total, int32_t zero_bias, int32_t *corr, int32_t *fix, int32_t *solve);

/* R99 of a multi-start run (Sec. III.A): p = the fraction of starts whose lowest
 * recorded energy (start_best, host [starts]) is <= e_target; the starts needed
 * for 99 % confidence n99 = ln(0.01) / ln(1 - p), at least 1 (1 when p >= 0.99),
 * not rounded; returns n99 * per_start (the total sample one start draws), or
 * -1 when no start reached e_target.  *p receives p (p may be NULL).  Host only. */
double spv_r99(const int64_t *start_best, int32_t starts, int64_t e_target, double per_start, double *p);

/*
 * Tree / degree-1 pre-processing (Sec. II.C): variables with at most one
 * neighbour (over couplers J != 0) are removed in rounds.  In each round every
 * remaining variable of degree <= 1 goes at once, except that of two variables
 * joined only to each other the larger index goes first.  Degree 0: fixed to
 * -sign(h) (+1 when h = 0).  Degree 1, neighbour j, coupler J: if |J| <= |h|
 * fixed to -sign(h) and J s is folded into h_j; otherwise inferred, s =
 * -sign(J) s_j, with -sign(J) h folded into h_j and -|J| into the offset.  The
 * remaining variables (index order) with their updated biases form the
 * reduced problem: E(s) = E'(s') + offset for every completion s of a reduced
 * state s' (spv_tree_complete).  All outputs are device arrays:
 *   kind [n]    0 remaining, 1 fixed, 2 inferred
 *   value [n]   the fixed value, or the factor f of an inferred s = f * s_parent
 *   parent [n]  the neighbour a removed degree-1 variable was folded into (-1: none)
 *   round [n]   the round of its removal (-1: remaining)
 *   order [n]   removed variables in removal order (rounds ascending)
 *   row_ptr [n+1], col [nnz], J [nnz], h [n], colour [n], orig_index [n]:
 *               the reduced problem (capacities of P)
 *   info [8]    int64: n_free, nnz_free, offset, n_fixed, n_inferred, rounds,
 *               0, n_removed
 * One workgroup; O(n + nnz) work.
 */
typedef struct {
    uint8_t *kind;
    int8_t *value;
    int32_t *parent;
    int32_t *round;
    int32_t *order;
    int32_t *row_ptr;
    int32_t *col;
    int32_t *J;
    int32_t *h;
    uint8_t *colour;
    int32_t *orig_index;
    int64_t *info;
} spv_tree_out;

spv_status spv_tree_reduce(spv_ctx *ctx, const spv_problem *P, const spv_tree_out *out, hipStream_t stream);

/* Completion of R reduced states reduced [R][n_free] (device) into full
 * states full [R][n] (device): the reduced variables, then the removed ones
 * in reverse removal order.  `t` is the output of spv_tree_reduce on a problem
 * of n variables; n_free and n_removed are its info[0] and info[7]. */
spv_status spv_tree_complete(spv_ctx *ctx, int32_t n, const spv_tree_out *t, int32_t n_free, int32_t n_removed,
                             const int8_t *reduced, int32_t R, int8_t *full, hipStream_t stream);

/*
 * Batched simulated annealing over B instances of uneven size (the residual
 * problems left after fixing, Sec. II.C / Sec. III.C) in ONE persistent
 * launch.  Work items (instance, block of 4*quads_per_item reads) are popped
 * from a device queue in largest-instance-first order; a workgroup reloads
 * an instance into LDS only when it changes.  Results are bit-identical to
 * spv_sample on each instance with the same schedule and seed, for every
 * launch shape.
 *   problems [B]  host array of device-resident problems; all share
 *                 scale_log2 (the threshold tables are common)
 *   betas [sweeps] host, shared schedule
 *   reads [B], seeds [B]  host
 *   spins [B], energies [B]  host arrays of device pointers ([reads][n] int8,
 *                 [reads] int64)
 *   opts          NULL for defaults.  threads / quads_per_item / wgs_per_cu
 *                 fix the shape (0 = default or tuned); flags:
 *                 SPV_BATCH_GRAPH captures the launch (descriptor upload,
 *                 queue reset, packing, persistent kernel) in a hipGraph,
 *                 cached per batch shape and replayed on later calls with the
 *                 same shape; SPV_BATCH_TUNE times candidate shapes on this
 *                 batch (short schedule) the first time a shape class is seen
 *                 and keeps the fastest on the context; SPV_BATCH_PAIRED with
 *                 threads (and wgs_per_cu) selects the paired body.
 * Two sampler bodies serve the batch.  The one-word body: an item is
 * (instance, block of quads_per_item quads), a lane holds one quad word of a
 * site.  The paired body (images of 4, 6 or 8 records per site on the
 * byte-parallel path; the default there): a lane holds both words of a pair of
 * quads of one site, and an item is (instance, k pairs) with k chosen per
 * instance so that k x class size fills the workgroup; the pairs share the
 * instance's records in LDS.  spv_batch_last_shape reports quads_per_item 0
 * for the paired body.  Both give the bits of one spv_sample per instance.
 * Descriptors are staged in pinned host memory; a call waits for the previous
 * batched launch on the context to finish reading them.
 */
#define SPV_BATCH_GRAPH 1u
#define SPV_BATCH_TUNE 2u
#define SPV_BATCH_PAIRED 4u
typedef struct {
    int32_t threads;
    int32_t quads_per_item;
    int32_t wgs_per_cu;
    uint32_t flags;
} spv_batch_opts;

spv_status spv_sample_batch(spv_ctx *ctx, int32_t B, const spv_problem *problems, const double *betas,
                            int32_t sweeps, const int32_t *reads, const uint64_t *seeds,
                            int8_t *const *spins, int64_t *const *energies, const spv_batch_opts *opts,
                            hipStream_t stream);

/* The launch shape the last spv_sample_batch call used (threads, quads per
 * item, workgroups per CU) and, when it was tuned, the best trial time in ms. */
spv_status spv_batch_last_shape(const spv_ctx *ctx, int32_t *threads, int32_t *quads_per_item,
                                int32_t *wgs_per_cu, float *tuned_ms);

/*
 * Serving loop: continuous batching of sample(+fix) requests of different
 * sizes.  A server owns `slots` execution slots, each a HIP stream with its own
 * scratch context.  A submitted request waits in a FIFO until a slot is free
 * and its LDS and HBM footprints fit the budgets left by the requests in
 * flight; it is then launched on the slot's stream and overlaps on the device
 * with the other in-flight requests.  A progress thread retires completed
 * requests (event query), timestamps them and admits waiting ones as capacity
 * frees up.  Results depend only on the request (counter-based randomness),
 * never on what else is in flight.
 *
 * Request kinds: SPV_REQ_SA (spv_sample), SPV_REQ_PT (spv_pt_sample, top-10
 * sample) and SPV_REQ_SQA (spv_sqa_sample).  With elite_frac > 0 the
 * persistence step (spv_persist_fix) runs on the produced sample (SA and SQA:
 * all reads; PT: the filled top-10 entries as assembled by spv_top_sample, once
 * the run has ended) into fix_out.
 * Every pointer in a request must stay valid until the request completes;
 * `betas` and `gammas` are copied at submission.
 * Slots are HIP streams; HIP spreads streams over GPU_MAX_HW_QUEUES hardware
 * queues (4 by default) and runs the kernels of one queue in order, so for
 * full overlap set that variable to at least `slots` before the HIP runtime
 * starts.
 */
typedef enum { SPV_REQ_SA = 1, SPV_REQ_PT = 2, SPV_REQ_SQA = 3 } spv_req_kind;

typedef struct {
    int32_t kind;
    spv_problem problem;
    uint64_t seed;
    const double *betas;  /* host: SA and SQA [sweeps], PT [K] */
    int32_t sweeps;
    int32_t reads;        /* SA, SQA */
    int8_t *spins;        /* SA, SQA: device [reads][n] */
    int64_t *energies;    /* SA, SQA: device [reads] */
    int32_t K, runs, chains, icm_lo, icm_hi; /* PT */
    spv_pt_out pt_out;    /* PT outputs; top_spins/top_E/top_count required for persistence */
    double elite_frac;    /* > 0 enables persistence */
    double threshold;
    int32_t gauge;
    spv_fix_out fix_out;
    const double *gammas; /* SQA: host [sweeps] */
    int32_t trotter;      /* SQA: slices per read */
} spv_request;

typedef struct {
    int32_t slots;        /* requests in flight at most (0 -> 8) */
    int64_t lds_budget;   /* LDS bytes (workgroups x LDS each) in flight (0 -> CUs x 160 KiB) */
    int64_t hbm_budget;   /* scratch bytes in flight (0 -> no limit) */
} spv_server_cfg;

typedef struct {
    int32_t status;       /* SPV_OK or the request's error (with persistence: also a
                             nonzero device status of the fixing step, fix_out.info[7]) */
    int64_t submit_ns;    /* host steady clock, nanoseconds */
    int64_t start_ns;     /* launched on a slot */
    int64_t done_ns;      /* completion observed */
    int32_t slot;
    int64_t lds_bytes;    /* footprint charged against the budgets while in flight */
    int64_t hbm_bytes;
} spv_result;

typedef struct spv_server spv_server;

spv_status spv_server_create(spv_ctx *ctx, const spv_server_cfg *cfg, spv_server **out);
/* Queues a request; SPV_EBUDGET if it alone exceeds a budget, SPV_EINVAL if malformed. */
spv_status spv_server_submit(spv_server *srv, const spv_request *req, uint64_t *ticket);
/* SPV_EAGAIN while the request is pending or running; else fills *res. */
spv_status spv_server_poll(spv_server *srv, uint64_t ticket, spv_result *res);
/* Blocks until the request completes and fills *res. */
spv_status spv_server_wait(spv_server *srv, uint64_t ticket, spv_result *res);
/* Blocks until nothing is queued or running. */
spv_status spv_server_drain(spv_server *srv);
/* Drains, stops the progress thread and releases the slots. */
void spv_server_destroy(spv_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SPVAR_H */
