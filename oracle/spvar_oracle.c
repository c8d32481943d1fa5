/*
 * spvar_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the hot path of multi-start
 * sample-persistence variable reduction (SPVAR, Sec. II, Algorithms 1 and 2):
 * the Monte Carlo samplers it calls (Metropolis simulated annealing, and
 * parallel tempering with isoenergetic cluster moves, Sec. III.A and
 * Sec. III.D.1) and the persistence step that fixes variables and reduces
 * the problem.  It exists to check the HIP library bit for bit.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.  It shares no code with the HIP library:
 * its Philox, acceptance tables, energies, persistence and reduction are
 * written here from the definitions below.
 *
 * Definitions (integer units; a real value is integer / 2^scale_log2):
 *
 *  Objective (Sec. I): E(s) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i, each
 *    undirected coupler counted once, minimised.
 *
 *  Metropolis update of spin i (Sec. III.A: SA; Sec. III.D.1: PT): local field
 *    f_i = h_i + sum_j J_ij s_j; x = -s_i f_i, so that flipping changes the
 *    energy by 2x.  x <= 0 always flips.  Otherwise x is written in base 512,
 *    x = sum_j d_j 512^j, and the flip is accepted iff every nonzero digit
 *    passes w_j < T_j[d_j] with T_j[d] = min(2^32-1,
 *    floor(2^32 * exp(-(beta * (2 * d * 512^j)) / 2^scale))).  The product of
 *    the digit factors is exp(-beta * 2x / 2^scale) up to 2^-32 rounding.
 *
 *  Sweep: colour classes in increasing colour, inside a class increasing
 *    index (classes are independent sets, so the in-class order is immaterial).
 *
 *  Random words, Philox4x32-10 with key (seed_lo, seed_hi):
 *    Metropolis digit j of (spin i, sweep t, replica r):
 *        Philox(i, t, r>>2, (2<<24)|j)[r&3]
 *    initial spin i of replica r: +1 iff Philox(i, 0, r>>2, 1<<24)[r&3] >> 31
 *    PT swap of pair (k,k+1) of chain-run c at sweep t, digit j:
 *        Philox(k, t, c, (3<<24)|(j>>2))[j&3]
 *    isoenergetic cluster move at slot k of run u at sweep t:
 *        Philox(k, t, u, 4<<24)[0]
 *
 *  PT replica exchange: pairs (k,k+1) with k = t (mod 2); D = E_k - E_{k+1};
 *    accept iff D <= 0 or the digit test of D passes with tables built for
 *    dbeta = beta_{k+1} - beta_k and unit 1 (T_j[d] uses d * 512^j); when
 *    D >= 512^nd with nd the smallest digit count whose next digit value has
 *    T == 0, the move is rejected (exactly what further digits would give).
 *
 *  Houdayer cluster move between chains 0 and 1 at slot k: q_i = s^A_i s^B_i;
 *    with n_neg sites at q=-1, the seed is the floor(w*n_neg/2^32)-th such
 *    site in index order; the cluster is its connected component among q=-1
 *    sites (edges with J != 0); the cluster is flipped in both replicas.
 *
 *  Top-10 sample (Sec. III.D.1): per slot of the colder half (the K/2
 *    coldest slots, k >= K - K/2) the 10
 *    lowest-energy distinct states seen after each sweep; insert iff fewer
 *    than 10 are held or E < the worst held; an identical state is never
 *    inserted twice; eviction removes the worst, latest-inserted among ties;
 *    output order (E, insertion).
 *
 *  Tempering checkpoint (continuing a run, Sec. III.D.1): a run resumed from
 *    the final states and top-10 lists of an earlier call, with sweep_offset
 *    advanced by that call's sweeps, is the same Markov chain under the same
 *    counter-based random words as one uninterrupted call: the slots start
 *    from the given states (a byte > 0 is +1, any other -1; energies are
 *    recomputed) and each list from its given entries, taken as inserted
 *    before any offer of the call in their listed order.  A list whose given
 *    count lies outside 0..10 starts empty and reports count -1.
 *
 *  Persistence (Algorithm 1): elite = first m = max(1, ceil(eps*R)) rows in
 *    (E, row) order; gauge (Sec. II.C zero-bias handling): classes of
 *    variables whose elite columns are equal up to a global sign, pivot p =
 *    lowest index of the largest class (ties: lower minimum index), elite
 *    rows multiplied by their value at p; c_i = sum_elite s_ri; fix iff
 *    |c_i| >= k_min = ceil(theta*m), to sign(c_i).
 *
 *  Reduction ("Update J and h", Algorithm 1): free set U in index order,
 *    J' = J[U,U], h'_u = h_u + sum_{j fixed} J_uj v_j,
 *    offset = sum_{i<j fixed} J_ij v_i v_j + sum_{i fixed} h_i v_i, so that
 *    E(s) = E'(s_U) + offset whenever s agrees with the fixed values.
 *
 *  Disconnected problems (Sec. II.C, special considerations): components of
 *    the graph whose edges are the couplers with J != 0, numbered in order of
 *    their smallest variable index.  Partial energy of component c in row r:
 *    E_c(r) = sum of J_ij s_i s_j over couplers inside c (each once) + sum of
 *    h_i s_i over i in c, so E(s) = sum_c E_c(s).  Recombination: the rows of
 *    each component are ordered by (E_c, row); merged row k takes, for every
 *    component, its variables from the k-th row in that component's order,
 *    and its energy is the sum over components of those k-th partial
 *    energies.  The best merged row therefore holds every component's best
 *    partial solution.
 *
 *  Multi-start SPVAR (Algorithm 2; zero-bias handling of Sec. II.C; sample
 *    split of the parameter appendix).  [Optional] the problem is tree
 *    pre-processed first (below).  Every start then runs stages on its own
 *    current problem; each stage samples that problem and records the
 *    energies in full-problem units (E' plus every offset above it), and the
 *    reductions follow one another:
 *      correlation step (corr_reads > 0; before the SPVAR step when
 *        corr_after == 0, the "pre-fixing" of the appendix, else after the
 *        SPVAR step and the tree step, the order the algorithm box lists):
 *        persistence with the gauge on, so the pivot's class of perfectly
 *        (anti)correlated variables is fixed, with the correlation elite
 *        fraction and threshold;
 *      SPVAR step (Algorithm 1): persistence with the caller's gauge mode,
 *        elite fraction and fixing threshold;
 *      [optional] tree pre-processing of the modified problem;
 *      solving step (solving_reads > 0): a sample of the modified problem,
 *        optionally recombined over its components as above.
 *    The first stage samples the problem every start shares: one sampler job
 *    with `seed`, start s owning reads [s*R, (s+1)*R).  The k-th later
 *    sampling stage (k = 1, 2) of start s uses seed + 1 + (k-1)*starts + s.
 *    The best state is the first minimum of the recorded energies in the
 *    order start 0 stage by stage, start 1, ...; it is lifted to the full
 *    problem through the reductions in reverse (fixed values; tree
 *    completion).  start_best[s] is the lowest energy start s recorded.
 *
 *  Simulated quantum annealing (Sec. III, "SQA": discrete-time path-integral
 *    Monte Carlo of the transverse-field Ising model, written from the
 *    Suzuki-Trotter mapping of Martonak, Santoro and Tosatti, Phys. Rev. B 66,
 *    094203 (2002)).  The paper names the sampler but not its parameters; the
 *    Trotter number P and the schedules beta_t, Gamma_t are the caller's.  P
 *    slices s^0..s^{P-1} per read form a ring; the effective energy in integer
 *    units is E_eff = sum_k E(s^k) - Jp_t sum_k sum_i s^k_i s^{(k+1) mod P}_i,
 *    sampled at inverse temperature beta_t / P, with Jp_t = round(P * Jperp *
 *    2^scale) (half away from zero) and Jperp = -ln(tanh(beta_t Gamma_t / P))
 *    / (2 beta_t), evaluated in double in exactly that order.  Updating spin i
 *    of slice k: g = f_i(s^k) - Jp_t (s^{k-1}_i + s^{k+1}_i), x = -s^k_i g, the
 *    digit test above with tables for beta_t / P.  A sweep visits the colour
 *    classes in order and, inside a class, the even slices and then the odd
 *    ones (each an independent set).  Slice k of read u is replica r = u P +
 *    (k mod 2) P/2 + floor(k/2) (even slices first), so its random words are
 *    Philox(i, t, r>>2, (6<<24)|j)[r&3] and its initial spins those of replica
 *    r above.  The sample of a read is its lowest-energy slice after the last
 *    sweep (ties: lowest k), with that slice's energy E.
 *
 *  Colour classes (the sweep's independent sets; not a step the paper states:
 *    the parallel sweep needs them).  Jones-Plassmann: vertex v has priority
 *    (word 0 of Philox(v, 0, 0, 5 << 24) under the seed, then v), higher
 *    first; in each round every uncoloured vertex whose priority exceeds that
 *    of all its uncoloured neighbours (every CSR entry is an edge) takes the
 *    smallest colour no coloured neighbour has.  The result equals first-fit
 *    greedy colouring in decreasing priority order.
 *
 *  Tree pre-processing (Sec. II.C): the degree of a remaining variable counts
 *    its couplers with J != 0 to remaining variables.  In every round all
 *    remaining variables of degree <= 1 are removed at once, except that of
 *    two remaining variables joined only to each other the larger index goes
 *    first.  Degree 0: fixed to -sign(h) (+1 when h = 0), offset += h s.
 *    Degree 1 with neighbour j and coupler J: if |J| <= |h| fixed to
 *    -sign(h), h_j += J s, offset += h s; else inferred s = -sign(J) s_j,
 *    h_j -= sign(J) h, offset -= |J|.  Rounds repeat until none is removed;
 *    the remaining variables (in index order) with their updated biases and
 *    the couplers among them form the reduced problem, so that E(s) =
 *    E'(s') + offset for every completion s of a reduced state s' (inferred
 *    values filled in from the last round back to the first).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#else
static int omp_get_thread_num(void) { return 0; }
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-4)
#define ORC_ENOMEM (-9)
#define ORC_EINTERNAL (-10)

#define TAG_INIT 1u
#define TAG_METRO 2u
#define TAG_SWAP 3u
#define TAG_ICM 4u
#define TAG_SQA 6u
#define DIGIT_BITS 9
#define DIGIT_SIZE 512
#define TOPK 10

typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *J;
    const int32_t *h;
    const uint8_t *colour;
    int32_t n_colours;
    int32_t scale_log2;
} orc_problem;

/* Parameters and outputs of the multi-start driver (definition above). */
typedef struct {
    const double *betas;      /* [sweeps] */
    int32_t sweeps;
    uint64_t seed;
    int32_t starts, corr_reads, fixing_reads, solving_reads;
    double elite_frac, threshold;
    int32_t gauge;
    double corr_elite_frac, corr_threshold;
    int32_t corr_after;       /* 0: correlation step before the SPVAR step, 1: after it (and the tree) */
    int32_t preprocess;       /* bit 0: tree before the loop; bit 1: tree after each SPVAR step */
    int32_t merge;
    int32_t sampler, trotter; /* 0 SA; 1 SQA over `trotter` slices with `gammas` */
    const double *gammas;
} orc_ms_params;

typedef struct {
    int64_t *corr_E, *fixing_E, *solving_E; /* [S][Rc], [S][F], [S][Rs] */
    uint8_t *fixed_mask;                    /* [S][n] */
    int8_t *fixed_val;                      /* [S][n] */
    int64_t *info;                          /* [S][8] */
    int64_t *info_pre;                      /* [8] */
    int64_t *start_best;                    /* [S] */
    int8_t *best_spins;                     /* [n] */
    int64_t *best_E;
} orc_ms_out;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two    */
/* 32x32->64 multiplications by fixed constants with a Weyl key schedule. */
/* ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t a = ctr[0], b = ctr[1], c = ctr[2], d = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)a;
        uint64_t pc = (uint64_t)0xCD9E8D57u * (uint64_t)c;
        uint32_t na = (uint32_t)(pc >> 32) ^ b ^ k0;
        uint32_t nb = (uint32_t)pc;
        uint32_t nc = (uint32_t)(pa >> 32) ^ d ^ k1;
        uint32_t nd = (uint32_t)pa;
        a = na; b = nb; c = nc; d = nd;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = a; out[1] = b; out[2] = c; out[3] = d;
}

/* Batch form for tests: out[i][0..3] = Philox(ctr[i][0..3], key). */
void orc_philox_batch(const uint32_t *ctr, const uint32_t key[2], uint32_t *out, int64_t count)
{
    int64_t i;
    for (i = 0; i < count; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint64_t seed, int which)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[which];
}

/* ---------------------------------------------------------------------- */
/* Objective (Sec. I).                                                     */
/* ---------------------------------------------------------------------- */
int64_t orc_energy(const orc_problem *P, const int8_t *s)
{
    int64_t e = 0;
    int32_t i, k;
    for (i = 0; i < P->n; ++i) {
        e += (int64_t)P->h[i] * s[i];
        for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
            int32_t j = P->col[k];
            if (j > i)
                e += (int64_t)P->J[k] * s[i] * s[j];
        }
    }
    return e;
}

void orc_energy_batch(const orc_problem *P, const int8_t *spins, int32_t R, int64_t *E)
{
    int32_t r;
    for (r = 0; r < R; ++r)
        E[r] = orc_energy(P, spins + (size_t)r * P->n);
}

static int64_t local_field(const orc_problem *P, const int8_t *s, int32_t i)
{
    int64_t f = P->h[i];
    int32_t k;
    for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
        f += (int64_t)P->J[k] * s[P->col[k]];
    return f;
}

/* Largest |h_i| + sum_j |J_ij|: bounds |x| of every Metropolis proposal. */
int64_t orc_x_max(const orc_problem *P)
{
    int64_t best = 0;
    int32_t i, k;
    for (i = 0; i < P->n; ++i) {
        int64_t v = llabs((long long)P->h[i]);
        for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
            v += llabs((long long)P->J[k]);
        if (v > best)
            best = v;
    }
    return best;
}

/* ---------------------------------------------------------------------- */
/* Integer acceptance thresholds.                                          */
/* ---------------------------------------------------------------------- */
uint32_t orc_threshold(double beta, int64_t unit, int32_t scale_log2, int32_t digit, uint32_t d)
{
    double X = (double)(unit * (int64_t)d * ((int64_t)1 << (DIGIT_BITS * digit)));
    double p = beta * X;
    double a = ldexp(p, -scale_log2);
    double v = exp(-a) * 4294967296.0;
    if (v >= 4294967295.0)
        return 0xFFFFFFFFu;
    return (uint32_t)floor(v);
}

static int32_t digits_for(int64_t xmax)
{
    int32_t nd = 1;
    while (nd < 7 && (xmax >> (DIGIT_BITS * nd)) != 0)
        ++nd;
    return nd;
}

/* Digit count of a swap test: the first digit position whose unit value
 * already has a zero threshold (capped at 7 digits = 63 bits). */
int32_t orc_swap_digits(double dbeta, int32_t scale_log2)
{
    int32_t nd;
    for (nd = 1; nd < 7; ++nd)
        if (orc_threshold(dbeta, 1, scale_log2, nd, 1) == 0)
            return nd;
    return 7;
}

/* Table for one beta: T[j*512 + d]. */
static void build_table(double beta, int64_t unit, int32_t scale_log2, int32_t nd, uint32_t *T)
{
    int32_t j, d;
    for (j = 0; j < nd; ++j)
        for (d = 0; d < DIGIT_SIZE; ++d)
            T[j * DIGIT_SIZE + d] = orc_threshold(beta, unit, scale_log2, j, (uint32_t)d);
}

/* ---------------------------------------------------------------------- */
/* Sweep order: colour classes ascending, inside a class index ascending.  */
/* ---------------------------------------------------------------------- */
static int32_t *default_order(const orc_problem *P)
{
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (P->n > 0 ? P->n : 1));
    int32_t pos = 0, c, i;
    if (!ord)
        return NULL;
    for (c = 0; c < P->n_colours; ++c)
        for (i = 0; i < P->n; ++i)
            if (P->colour[i] == c)
                ord[pos++] = i;
    if (pos != P->n) {
        free(ord);
        return NULL;
    }
    return ord;
}

/* One Metropolis sweep of one replica; returns the energy change. */
static int64_t metropolis_sweep(const orc_problem *P, const int32_t *order, int8_t *s,
                                const uint32_t *T, int32_t nd, uint32_t t, uint32_t r,
                                uint64_t seed)
{
    int64_t dE = 0;
    int32_t p;
    for (p = 0; p < P->n; ++p) {
        int32_t i = order[p];
        int64_t f = local_field(P, s, i);
        int64_t x = -(int64_t)s[i] * f;
        int accept = 1;
        if (x > 0) {
            int32_t j;
            for (j = 0; j < nd && accept; ++j) {
                uint32_t d = (uint32_t)((x >> (DIGIT_BITS * j)) & (DIGIT_SIZE - 1));
                if (d != 0) {
                    uint32_t w = philox_word((uint32_t)i, t, r >> 2,
                                             (TAG_METRO << 24) | (uint32_t)j, seed, (int)(r & 3));
                    if (!(w < T[j * DIGIT_SIZE + d]))
                        accept = 0;
                }
            }
        }
        if (accept) {
            s[i] = (int8_t)(-s[i]);
            dE += 2 * x;
        }
    }
    return dE;
}

static void init_spins(int32_t n, uint32_t r, uint64_t seed, int8_t *s)
{
    int32_t i;
    for (i = 0; i < n; ++i) {
        uint32_t w = philox_word((uint32_t)i, 0, r >> 2, TAG_INIT << 24, seed, (int)(r & 3));
        s[i] = (w >> 31) ? 1 : -1;
    }
}

static int check_problem(const orc_problem *P)
{
    int32_t i;
    if (!P || P->n < 0 || P->n_colours < 1 || P->n_colours > 255)
        return ORC_EINVAL;
    for (i = 0; i < P->n; ++i)
        if (P->colour[i] >= P->n_colours)
            return ORC_EINVAL;
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Simulated annealing: one Metropolis sweep per entry of betas.           */
/* Reads r in [r_begin, r_end); outputs are indexed from r_begin.          */
/* order: optional visit order (must list classes in increasing colour).  */
/* ---------------------------------------------------------------------- */
int orc_sa_sample(const orc_problem *P, const double *betas, int32_t sweeps, uint64_t seed,
                  uint32_t sweep_offset, int32_t r_begin, int32_t r_end, const int8_t *init,
                  const int32_t *order_in, int8_t *spins_out, int64_t *E_out)
{
    int32_t nd, t, r;
    uint32_t *tables;
    int32_t *order;
    int rc = check_problem(P);
    if (rc)
        return rc;
    if (sweeps < 0 || r_begin < 0 || r_end < r_begin)
        return ORC_EINVAL;
    for (t = 0; t < sweeps; ++t)
        if (!(betas[t] >= 0.0) || isinf(betas[t]))
            return ORC_EINVAL;
    nd = digits_for(orc_x_max(P));
    tables = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(sweeps > 0 ? sweeps : 1) * nd * DIGIT_SIZE);
    if (order_in) {
        order = (int32_t *)malloc(sizeof(int32_t) * (P->n > 0 ? P->n : 1));
        if (order)
            memcpy(order, order_in, sizeof(int32_t) * P->n);
    } else {
        order = default_order(P);
    }
    if (!tables || !order) {
        free(tables);
        free(order);
        return ORC_ENOMEM;
    }
    for (t = 0; t < sweeps; ++t)
        build_table(betas[t], 2, P->scale_log2, nd, tables + (size_t)t * nd * DIGIT_SIZE);
    for (r = r_begin; r < r_end; ++r) {
        int8_t *s = spins_out + (size_t)(r - r_begin) * P->n;
        int64_t E;
        if (init)
            memcpy(s, init + (size_t)(r - r_begin) * P->n, (size_t)P->n);
        else
            init_spins(P->n, (uint32_t)r, seed, s);
        E = orc_energy(P, s);
        for (t = 0; t < sweeps; ++t)
            E += metropolis_sweep(P, order, s, tables + (size_t)t * nd * DIGIT_SIZE, nd,
                                  sweep_offset + (uint32_t)t, (uint32_t)r, seed);
        if (E != orc_energy(P, s)) {
            free(tables);
            free(order);
            return ORC_EINTERNAL;
        }
        E_out[r - r_begin] = E;
    }
    free(tables);
    free(order);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Simulated quantum annealing (path-integral Monte Carlo over P slices).  */
/* ---------------------------------------------------------------------- */
/* Inter-slice coupling of one sweep in integer units (see the header). */
int orc_sqa_coupling(double beta, double gamma, int32_t trotter, int32_t scale_log2, int64_t *jp)
{
    double arg, jperp, v;
    if (!(beta > 0.0) || !(gamma > 0.0) || isinf(beta) || isinf(gamma) || trotter < 1)
        return ORC_EINVAL;
    arg = beta * gamma / (double)trotter;
    jperp = -0.5 * log(tanh(arg)) / beta;
    v = jperp * (double)trotter * ldexp(1.0, scale_log2);
    if (!(v >= 0.0) || !(v < 16777216.0))
        return ORC_ERANGE;
    *jp = (int64_t)floor(v + 0.5);
    return ORC_OK;
}

/* Replica index of slice k of read u (even slices first). */
static uint32_t sqa_replica(int32_t u, int32_t k, int32_t trotter)
{
    return (uint32_t)((int64_t)u * trotter + (int64_t)(k & 1) * (trotter / 2) + (k >> 1));
}

/* Reads u in [r_begin, r_end): slices_out [R][P][n] and Ecl_out [R][P] hold
 * every slice after the last sweep (either may be NULL); spins_out [R][n],
 * E_out [R] and best_out [R] the sample (lowest-energy slice). */
int orc_sqa_sample(const orc_problem *P, const double *betas, const double *gammas, int32_t sweeps,
                   int32_t trotter, uint64_t seed, int32_t r_begin, int32_t r_end, int8_t *slices_out,
                   int64_t *Ecl_out, int8_t *spins_out, int64_t *E_out, int32_t *best_out)
{
    int32_t nd, t, u, k, c, par, i, j;
    int64_t jmax = 0, *jp;
    uint32_t *tables;
    int8_t *s;
    const int32_t n = P ? P->n : 0;
    int rc = check_problem(P);
    if (rc)
        return rc;
    if (sweeps < 0 || trotter < 2 || (trotter & 1) || r_begin < 0 || r_end < r_begin)
        return ORC_EINVAL;
    jp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sweeps > 0 ? sweeps : 1));
    if (!jp)
        return ORC_ENOMEM;
    for (t = 0; t < sweeps; ++t) {
        rc = orc_sqa_coupling(betas[t], gammas[t], trotter, P->scale_log2, &jp[t]);
        if (rc) {
            free(jp);
            return rc;
        }
        if (jp[t] > jmax)
            jmax = jp[t];
    }
    nd = digits_for(orc_x_max(P) + 2 * jmax);
    tables = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(sweeps > 0 ? sweeps : 1) * nd * DIGIT_SIZE);
    s = (int8_t *)malloc((size_t)trotter * (n > 0 ? n : 1));
    if (!tables || !s) {
        free(jp);
        free(tables);
        free(s);
        return ORC_ENOMEM;
    }
    for (t = 0; t < sweeps; ++t)
        build_table(betas[t] / (double)trotter, 2, P->scale_log2, nd, tables + (size_t)t * nd * DIGIT_SIZE);
    for (u = r_begin; u < r_end; ++u) {
        int64_t bestE = 0;
        int32_t best = 0;
        for (k = 0; k < trotter; ++k)
            init_spins(n, sqa_replica(u, k, trotter), seed, s + (size_t)k * n);
        for (t = 0; t < sweeps; ++t) {
            const uint32_t *T = tables + (size_t)t * nd * DIGIT_SIZE;
            for (c = 0; c < P->n_colours; ++c)
                for (par = 0; par < 2; ++par)
                    for (i = 0; i < n; ++i) {
                        if (P->colour[i] != c)
                            continue;
                        for (k = par; k < trotter; k += 2) {
                            int8_t *sk = s + (size_t)k * n;
                            const int8_t up = s[(size_t)((k + trotter - 1) % trotter) * n + i];
                            const int8_t dn = s[(size_t)((k + 1) % trotter) * n + i];
                            const int64_t g = local_field(P, sk, i) - jp[t] * (int64_t)(up + dn);
                            const int64_t x = -(int64_t)sk[i] * g;
                            const uint32_t r = sqa_replica(u, k, trotter);
                            int accept = 1;
                            if (x > 0)
                                for (j = 0; j < nd && accept; ++j) {
                                    uint32_t d = (uint32_t)((x >> (DIGIT_BITS * j)) & (DIGIT_SIZE - 1));
                                    if (d != 0) {
                                        uint32_t w = philox_word((uint32_t)i, (uint32_t)t, r >> 2,
                                                                 (TAG_SQA << 24) | (uint32_t)j, seed, (int)(r & 3));
                                        if (!(w < T[j * DIGIT_SIZE + d]))
                                            accept = 0;
                                    }
                                }
                            if (accept)
                                sk[i] = (int8_t)(-sk[i]);
                        }
                    }
        }
        for (k = 0; k < trotter; ++k) {
            const int64_t E = orc_energy(P, s + (size_t)k * n);
            if (Ecl_out)
                Ecl_out[(size_t)(u - r_begin) * trotter + k] = E;
            if (k == 0 || E < bestE) {
                bestE = E;
                best = k;
            }
        }
        if (slices_out)
            memcpy(slices_out + (size_t)(u - r_begin) * trotter * n, s, (size_t)trotter * n);
        memcpy(spins_out + (size_t)(u - r_begin) * n, s + (size_t)best * n, (size_t)n);
        E_out[u - r_begin] = bestE;
        best_out[u - r_begin] = best;
    }
    free(jp);
    free(tables);
    free(s);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Parallel tempering (+ Houdayer cluster moves, + top-10 sample).         */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t E[TOPK];
    int64_t when[TOPK];
    int32_t count;
    int8_t *state; /* [TOPK][n] */
} topk_list;

static void topk_offer(topk_list *L, int32_t n, int64_t E, const int8_t *s, int64_t when)
{
    int32_t e, victim;
    if (L->count == TOPK) {
        int64_t worst = L->E[0];
        for (e = 1; e < TOPK; ++e)
            if (L->E[e] > worst)
                worst = L->E[e];
        if (!(E < worst))
            return;
    }
    for (e = 0; e < L->count; ++e)
        if (L->E[e] == E && memcmp(L->state + (size_t)e * n, s, (size_t)n) == 0)
            return;
    if (L->count < TOPK) {
        victim = L->count++;
    } else {
        victim = 0;
        for (e = 1; e < TOPK; ++e)
            if (L->E[e] > L->E[victim] || (L->E[e] == L->E[victim] && L->when[e] > L->when[victim]))
                victim = e;
    }
    L->E[victim] = E;
    L->when[victim] = when;
    memcpy(L->state + (size_t)victim * n, s, (size_t)n);
}

/* Houdayer move on replicas A and B; returns 1 if a cluster was flipped. */
static int icm_move(const orc_problem *P, int8_t *A, int8_t *B, int64_t *EA, int64_t *EB,
                    uint32_t w, int32_t *queue, uint8_t *in_cluster)
{
    int32_t n = P->n, i, k, n_neg = 0, target, seed_site = -1, head = 0, tail = 0;
    int64_t dA = 0, dB = 0;
    for (i = 0; i < n; ++i)
        if (A[i] != B[i])
            ++n_neg;
    if (n_neg == 0)
        return 0;
    target = (int32_t)(((uint64_t)w * (uint64_t)n_neg) >> 32);
    for (i = 0; i < n; ++i) {
        if (A[i] != B[i]) {
            if (target == 0) {
                seed_site = i;
                break;
            }
            --target;
        }
    }
    memset(in_cluster, 0, (size_t)n);
    in_cluster[seed_site] = 1;
    queue[tail++] = seed_site;
    while (head < tail) {
        int32_t v = queue[head++];
        for (k = P->row_ptr[v]; k < P->row_ptr[v + 1]; ++k) {
            int32_t u = P->col[k];
            if (P->J[k] != 0 && A[u] != B[u] && !in_cluster[u]) {
                in_cluster[u] = 1;
                queue[tail++] = u;
            }
        }
    }
    /* Energy change of flipping the cluster C: bias terms of C and couplers
     * crossing the cluster boundary change sign. */
    for (head = 0; head < tail; ++head) {
        int32_t v = queue[head];
        dA += -2 * (int64_t)P->h[v] * A[v];
        dB += -2 * (int64_t)P->h[v] * B[v];
        for (k = P->row_ptr[v]; k < P->row_ptr[v + 1]; ++k) {
            int32_t u = P->col[k];
            if (!in_cluster[u]) {
                dA += -2 * (int64_t)P->J[k] * A[v] * A[u];
                dB += -2 * (int64_t)P->J[k] * B[v] * B[u];
            }
        }
    }
    for (head = 0; head < tail; ++head) {
        int32_t v = queue[head];
        A[v] = (int8_t)(-A[v]);
        B[v] = (int8_t)(-B[v]);
    }
    *EA += dA;
    *EB += dB;
    return 1;
}

/* Test hook: one Houdayer move with a given random word.  cluster[n] is set
 * to 1 on the flipped sites.  Returns 1 if a cluster was flipped. */
int orc_icm_step(const orc_problem *P, int8_t *A, int8_t *B, int64_t *EA, int64_t *EB,
                 uint32_t w, uint8_t *cluster)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P->n > 0 ? P->n : 1));
    int rc;
    if (!queue)
        return ORC_ENOMEM;
    memset(cluster, 0, (size_t)P->n);
    rc = icm_move(P, A, B, EA, EB, w, queue, cluster);
    free(queue);
    return rc;
}

static int swap_accept(int64_t D, const uint32_t *T, int32_t nd, uint32_t k, uint32_t t,
                       uint32_t c, uint64_t seed)
{
    int32_t j;
    if (D <= 0)
        return 1;
    if (nd < 7 && (D >> (DIGIT_BITS * nd)) != 0)
        return 0;
    for (j = 0; j < nd; ++j) {
        uint32_t d = (uint32_t)((D >> (DIGIT_BITS * j)) & (DIGIT_SIZE - 1));
        if (d != 0) {
            uint32_t w = philox_word(k, t, c, (TAG_SWAP << 24) | ((uint32_t)j >> 2), seed, j & 3);
            if (!(w < T[j * DIGIT_SIZE + d]))
                return 0;
        }
    }
    return 1;
}

/* Test hook: the replica-exchange decision for an energy difference D. */
int orc_swap_test(int64_t D, double dbeta, int32_t scale_log2, uint32_t k, uint32_t t, uint32_t c,
                  uint64_t seed)
{
    uint32_t T[7 * DIGIT_SIZE];
    int32_t nd = orc_swap_digits(dbeta, scale_log2);
    build_table(dbeta, 1, scale_log2, nd, T);
    return swap_accept(D, T, nd, k, t, c, seed);
}

/*
 * runs [run_begin, run_end) of a PT job with K slots (betas ascending) and
 * `chains` independent ladders per run.  Outputs are indexed from run_begin:
 *   final_spins [runs][chains][K][n], final_E [runs][chains][K]   (optional)
 *   top_spins [runs][chains][K/2][10][n], top_E [..][10], top_count [..]
 *     (optional; unfilled entries: E = INT64_MAX, spins 0)
 *   log_E [sweeps][chains][K], log_spins [sweeps][chains][K][n]  (optional,
 *     only for run_begin: the state after every sweep, for tests)
 * icm_lo..icm_hi: slot window of the cluster moves (needs chains == 2).
 */
/* Host threads that share one tempering run (1: sequential).  Inside a sweep the
 * slots' Metropolis sweeps, the cluster moves of the K slot pairs and the top-10
 * offers of the lists touch disjoint replicas and lists, so spreading them over
 * threads leaves every replica's own sequence of updates, and so the result,
 * unchanged; the replica exchange stays sequential. */
static int32_t g_slot_threads = 1;

void orc_set_slot_threads(int32_t threads)
{
    g_slot_threads = threads < 1 ? 1 : threads;
}

int orc_pt_sample(const orc_problem *P, const double *betas, int32_t K, int32_t runs,
                  int32_t chains, int32_t sweeps, uint64_t seed, uint32_t sweep_offset,
                  int32_t icm_lo, int32_t icm_hi, int32_t run_begin, int32_t run_end,
                  int8_t *final_spins, int64_t *final_E, int8_t *top_spins, int64_t *top_E,
                  int32_t *top_count, int64_t *log_E, int8_t *log_spins, const int8_t *resume_spins,
                  const int8_t *resume_top_spins, const int64_t *resume_top_E,
                  const int32_t *resume_top_count)
{
    int32_t n = P->n, nd, k, run, ch, ls, half = K / 2;
    int32_t nrep = chains * K, nth = g_slot_threads;
    uint32_t *mtab = NULL, *stab = NULL;
    int32_t *snd = NULL, *order = NULL, *queue = NULL;
    int8_t *S = NULL, *tmp = NULL;
    uint8_t *inc = NULL;
    int64_t *E = NULL;
    topk_list *lists = NULL;
    uint8_t *bad = NULL; /* per list: its checkpoint count was outside 0..10 */
    int rc = check_problem(P);
    if (rc)
        return rc;
    if (K < 1 || runs < 1 || chains < 1 || sweeps < 0 || run_begin < 0 || run_end > runs ||
        run_end < run_begin)
        return ORC_EINVAL;
    if (icm_hi > icm_lo && (chains != 2 || icm_lo < 0 || icm_hi > K))
        return ORC_EINVAL;
    if ((resume_top_count != NULL) != (resume_top_E != NULL) ||
        (resume_top_count != NULL) != (resume_top_spins != NULL))
        return ORC_EINVAL;
    for (k = 0; k < K; ++k) {
        if (!(betas[k] >= 0.0) || isinf(betas[k]))
            return ORC_EINVAL;
        if (k > 0 && betas[k] < betas[k - 1])
            return ORC_EINVAL;
    }
    nd = digits_for(orc_x_max(P));
    mtab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K * nd * DIGIT_SIZE);
    stab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K * 7 * DIGIT_SIZE);
    snd = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    order = default_order(P);
    queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)nth * (n > 0 ? n : 1)); /* one per thread */
    inc = (uint8_t *)malloc((size_t)nth * (n > 0 ? n : 1));
    S = (int8_t *)malloc((size_t)nrep * (n > 0 ? n : 1));
    tmp = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    E = (int64_t *)malloc(sizeof(int64_t) * (size_t)nrep);
    lists = (topk_list *)calloc((size_t)chains * (half > 0 ? half : 1), sizeof(topk_list));
    bad = (uint8_t *)calloc((size_t)chains * (half > 0 ? half : 1), 1);
    if (!mtab || !stab || !snd || !order || !queue || !inc || !S || !tmp || !E || !lists || !bad) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (k = 0; k < chains * half; ++k) {
        lists[k].state = (int8_t *)malloc((size_t)TOPK * (n > 0 ? n : 1));
        if (!lists[k].state) {
            rc = ORC_ENOMEM;
            goto done;
        }
    }
    for (k = 0; k < K; ++k)
        build_table(betas[k], 2, P->scale_log2, nd, mtab + (size_t)k * nd * DIGIT_SIZE);
    for (k = 0; k + 1 < K; ++k) {
        double db = betas[k + 1] - betas[k];
        snd[k] = orc_swap_digits(db, P->scale_log2);
        build_table(db, 1, P->scale_log2, snd[k], stab + (size_t)k * 7 * DIGIT_SIZE);
    }
    for (run = run_begin; run < run_end; ++run) {
        int32_t lr = run - run_begin;
        int64_t when = 0;
        for (ch = 0; ch < chains * half; ++ch) {
            topk_list *L = &lists[ch];
            size_t base = ((size_t)lr * chains * half + ch) * TOPK;
            int32_t c = resume_top_count ? resume_top_count[(size_t)lr * chains * half + ch] : 0;
            int32_t e, i;
            L->count = 0;
            bad[ch] = c < 0 || c > TOPK;
            if (bad[ch] || !resume_top_count)
                continue;
            /* checkpoint entries count as inserted before this call, in list order */
            for (e = 0; e < c; ++e) {
                L->E[e] = resume_top_E[base + e];
                L->when[e] = (int64_t)e - TOPK;
                for (i = 0; i < n; ++i)
                    L->state[(size_t)e * n + i] = resume_top_spins[(base + e) * n + i] > 0 ? 1 : -1;
            }
            L->count = c;
        }
        for (ch = 0; ch < chains; ++ch)
            for (k = 0; k < K; ++k) {
                uint32_t r = (uint32_t)((run * chains + ch) * K + k);
                int8_t *s = S + (size_t)(ch * K + k) * n;
                if (resume_spins) {
                    const int8_t *from = resume_spins + ((size_t)lr * nrep + ch * K + k) * n;
                    int32_t i;
                    for (i = 0; i < n; ++i)
                        s[i] = from[i] > 0 ? 1 : -1;
                } else {
                    init_spins(n, r, seed, s);
                }
                E[ch * K + k] = orc_energy(P, s);
            }
        for (ls = 0; ls < sweeps; ++ls) {
            uint32_t t = sweep_offset + (uint32_t)ls;
            /* 1. Metropolis on every slot. */
            {
                int32_t x;
#pragma omp parallel for num_threads(nth) schedule(static) if (nth > 1)
                for (x = 0; x < nrep; ++x) {
                    int32_t xc = x / K, xk = x % K;
                    uint32_t r = (uint32_t)((run * chains + xc) * K + xk);
                    E[x] += metropolis_sweep(P, order, S + (size_t)x * n, mtab + (size_t)xk * nd * DIGIT_SIZE, nd,
                                             t, r, seed);
                }
            }
            /* 2. Replica exchange inside each chain. */
            for (ch = 0; ch < chains; ++ch) {
                uint32_t c = (uint32_t)(run * chains + ch);
                for (k = (int32_t)(t & 1u); k + 1 < K; k += 2) {
                    int64_t D = E[ch * K + k] - E[ch * K + k + 1];
                    if (swap_accept(D, stab + (size_t)k * 7 * DIGIT_SIZE, snd[k], (uint32_t)k, t, c,
                                    seed)) {
                        int8_t *a = S + (size_t)(ch * K + k) * n;
                        int8_t *b = S + (size_t)(ch * K + k + 1) * n;
                        int64_t e = E[ch * K + k];
                        memcpy(tmp, a, (size_t)n);
                        memcpy(a, b, (size_t)n);
                        memcpy(b, tmp, (size_t)n);
                        E[ch * K + k] = E[ch * K + k + 1];
                        E[ch * K + k + 1] = e;
                    }
                }
            }
            /* 3. Isoenergetic cluster moves between the two chains. */
            {
                int32_t x;
#pragma omp parallel for num_threads(nth) schedule(dynamic) if (nth > 1)
                for (x = icm_lo; x < icm_hi; ++x) {
                    size_t tid = (size_t)omp_get_thread_num();
                    uint32_t w = philox_word((uint32_t)x, t, (uint32_t)run, TAG_ICM << 24, seed, 0);
                    icm_move(P, S + (size_t)x * n, S + (size_t)(K + x) * n, &E[x], &E[K + x], w,
                             queue + tid * (size_t)n, inc + tid * (size_t)n);
                }
            }
            /* 4. Offer the colder half to the top-10 lists (offer numbers in (chain, slot) order). */
            {
                int32_t x;
#pragma omp parallel for num_threads(nth) schedule(static) if (nth > 1)
                for (x = 0; x < chains * half; ++x) {
                    int32_t xc = x / half, xk = K - half + x % half;
                    topk_offer(&lists[x], n, E[xc * K + xk], S + (size_t)(xc * K + xk) * n, when + x);
                }
                when += chains * half;
            }
            if (log_E && run == run_begin) {
                memcpy(log_E + (size_t)ls * nrep, E, sizeof(int64_t) * (size_t)nrep);
                if (log_spins)
                    memcpy(log_spins + (size_t)ls * nrep * n, S, (size_t)nrep * n);
            }
        }
        for (k = 0; k < nrep; ++k)
            if (E[k] != orc_energy(P, S + (size_t)k * n)) {
                rc = ORC_EINTERNAL;
                goto done;
            }
        if (final_spins)
            memcpy(final_spins + (size_t)lr * nrep * n, S, (size_t)nrep * n);
        if (final_E)
            memcpy(final_E + (size_t)lr * nrep, E, sizeof(int64_t) * (size_t)nrep);
        if (top_E) {
            for (ch = 0; ch < chains * half; ++ch) {
                topk_list *L = &lists[ch];
                size_t base = ((size_t)lr * chains * half + ch) * TOPK;
                int32_t rank, e;
                uint8_t used[TOPK] = {0};
                for (rank = 0; rank < TOPK; ++rank) {
                    int32_t best = -1;
                    for (e = 0; e < L->count; ++e)
                        if (!used[e] && (best < 0 || L->E[e] < L->E[best] ||
                                         (L->E[e] == L->E[best] && L->when[e] < L->when[best])))
                            best = e;
                    if (best < 0) {
                        top_E[base + rank] = INT64_MAX;
                        if (top_spins)
                            memset(top_spins + (base + rank) * n, 0, (size_t)n);
                        continue;
                    }
                    used[best] = 1;
                    top_E[base + rank] = L->E[best];
                    if (top_spins)
                        memcpy(top_spins + (base + rank) * n, L->state + (size_t)best * n, (size_t)n);
                }
                if (top_count)
                    top_count[(size_t)lr * chains * half + ch] = bad[ch] ? -1 : L->count;
            }
        }
    }
done:
    if (lists)
        for (k = 0; k < chains * half; ++k)
            free(lists[k].state);
    free(lists);
    free(bad);
    free(E);
    free(tmp);
    free(S);
    free(inc);
    free(queue);
    free(order);
    free(snd);
    free(stab);
    free(mtab);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Persistence and reduction (Algorithm 1).                                */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t E;
    int32_t row;
} elite_key;

static int cmp_elite(const void *a, const void *b)
{
    const elite_key *x = (const elite_key *)a, *y = (const elite_key *)b;
    if (x->E != y->E)
        return x->E < y->E ? -1 : 1;
    return (x->row > y->row) - (x->row < y->row);
}

typedef struct {
    const int8_t *col; /* canonical column, m entries */
    int32_t m;
    int32_t idx;
} canon_key;

static int cmp_canon(const void *a, const void *b)
{
    const canon_key *x = (const canon_key *)a, *y = (const canon_key *)b;
    int c = memcmp(x->col, y->col, (size_t)x->m);
    if (c)
        return c;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/*
 * info[8]: n_free, nnz_free, offset, n_fixed, pivot (-1 without gauge), m, k_min, 0.
 * gauge: 0 off, 1 on, 2 on iff every h_i == 0.
 * The reduced CSR buffers must hold n (rows) and nnz (entries).
 */
int orc_persist_fix(const orc_problem *P, const int8_t *samples, const int64_t *energies,
                    int32_t R, double elite_frac, double threshold, int32_t gauge,
                    uint8_t *fixed_mask, int8_t *fixed_val, int32_t *row_ptr_o, int32_t *col_o,
                    int32_t *J_o, int32_t *h_o, uint8_t *colour_o, int32_t *orig_o, int64_t *info)
{
    int32_t n = P->n, i, k, r, m, kmin, pivot = -1, use_gauge = 0;
    int32_t *elite = NULL, *newid = NULL;
    elite_key *idx = NULL;
    int8_t *g = NULL, *canon = NULL;
    int64_t *cnt = NULL, offset = 0;
    int32_t n_free = 0, nnz_free = 0, n_fixed = 0;
    double mm, kk;
    int rc = check_problem(P);
    if (rc)
        return rc;
    if (R < 1 || !(elite_frac > 0.0 && elite_frac <= 1.0) || !(threshold > 0.0 && threshold <= 1.0) ||
        gauge < 0 || gauge > 2)
        return ORC_EINVAL;
    for (r = 0; r < R; ++r)
        for (i = 0; i < n; ++i)
            if (samples[(size_t)r * n + i] != 1 && samples[(size_t)r * n + i] != -1)
                return ORC_EINVAL;
    /* INT64_MIN is no energy of any state (|E| <= sum|J| + sum|h|): it marks an invalid read. */
    for (r = 0; r < R; ++r)
        if (energies[r] == INT64_MIN)
            return ORC_EINVAL;
    mm = ceil(elite_frac * (double)R);
    m = (int32_t)mm;
    if (m < 1)
        m = 1;
    if (m > R)
        m = R;
    kk = ceil(threshold * (double)m);
    kmin = (int32_t)kk;
    if (kmin < 1)
        return ORC_EINVAL;
    idx = (elite_key *)malloc(sizeof(elite_key) * (size_t)R);
    elite = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    g = (int8_t *)malloc((size_t)m);
    cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    newid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!idx || !elite || !g || !cnt || !newid) {
        rc = ORC_ENOMEM;
        goto done;
    }
    /* Elite: the m lowest (E, row) rows; kept in row order. */
    for (r = 0; r < R; ++r) {
        idx[r].E = energies[r];
        idx[r].row = r;
    }
    qsort(idx, (size_t)R, sizeof(elite_key), cmp_elite);
    for (r = 0; r < m; ++r)
        elite[r] = idx[r].row;
    {
        int32_t a, b;
        for (a = 1; a < m; ++a) { /* insertion sort by row */
            int32_t v = elite[a];
            for (b = a - 1; b >= 0 && elite[b] > v; --b)
                elite[b + 1] = elite[b];
            elite[b + 1] = v;
        }
    }
    if (gauge == 1)
        use_gauge = 1;
    else if (gauge == 2) {
        use_gauge = 1;
        for (i = 0; i < n; ++i)
            if (P->h[i] != 0)
                use_gauge = 0;
    }
    for (r = 0; r < m; ++r)
        g[r] = 1;
    if (use_gauge && n > 0) {
        /* Canonical column of i: its elite values times its value in the
         * first elite row; equal canonical columns <=> columns equal up to
         * a global sign. */
        canon_key *cols = (canon_key *)malloc(sizeof(canon_key) * (size_t)n);
        int32_t best_size = 0, best_min = 0, a = 0;
        canon = (int8_t *)malloc((size_t)n * m);
        if (!cols || !canon) {
            free(cols);
            rc = ORC_ENOMEM;
            goto done;
        }
        for (i = 0; i < n; ++i) {
            int8_t first = samples[(size_t)elite[0] * n + i];
            for (r = 0; r < m; ++r)
                canon[(size_t)i * m + r] = (int8_t)(samples[(size_t)elite[r] * n + i] * first);
            cols[i].col = canon + (size_t)i * m;
            cols[i].m = m;
            cols[i].idx = i;
        }
        qsort(cols, (size_t)n, sizeof(canon_key), cmp_canon);
        while (a < n) {
            int32_t b = a + 1, mn = cols[a].idx;
            while (b < n && memcmp(cols[a].col, cols[b].col, (size_t)m) == 0) {
                if (cols[b].idx < mn)
                    mn = cols[b].idx;
                ++b;
            }
            if (b - a > best_size || (b - a == best_size && mn < best_min)) {
                best_size = b - a;
                best_min = mn;
            }
            a = b;
        }
        pivot = best_min;
        for (r = 0; r < m; ++r)
            g[r] = samples[(size_t)elite[r] * n + pivot];
        free(cols);
    }
    for (r = 0; r < m; ++r)
        for (i = 0; i < n; ++i)
            cnt[i] += (int64_t)g[r] * samples[(size_t)elite[r] * n + i];
    for (i = 0; i < n; ++i) {
        int64_t c = cnt[i];
        if (llabs((long long)c) >= kmin) {
            fixed_mask[i] = 1;
            fixed_val[i] = (int8_t)(c > 0 ? 1 : -1);
            ++n_fixed;
        } else {
            fixed_mask[i] = 0;
            fixed_val[i] = 0;
        }
    }
    /* Reduction. */
    for (i = 0; i < n; ++i)
        newid[i] = fixed_mask[i] ? -1 : n_free++;
    row_ptr_o[0] = 0;
    for (i = 0; i < n; ++i) {
        if (fixed_mask[i]) {
            offset += (int64_t)P->h[i] * fixed_val[i];
            for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
                int32_t j = P->col[k];
                if (j > i && fixed_mask[j])
                    offset += (int64_t)P->J[k] * fixed_val[i] * fixed_val[j];
            }
        } else {
            int32_t u = newid[i];
            int64_t hv = P->h[i];
            for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
                int32_t j = P->col[k];
                if (fixed_mask[j]) {
                    hv += (int64_t)P->J[k] * fixed_val[j];
                } else {
                    col_o[nnz_free] = newid[j];
                    J_o[nnz_free] = P->J[k];
                    ++nnz_free;
                }
            }
            if (hv > INT32_MAX || hv < INT32_MIN) {
                rc = ORC_ERANGE;
                goto done;
            }
            h_o[u] = (int32_t)hv;
            colour_o[u] = P->colour[i];
            orig_o[u] = i;
            row_ptr_o[u + 1] = nnz_free;
        }
    }
    info[0] = n_free;
    info[1] = nnz_free;
    info[2] = offset;
    info[3] = n_fixed;
    info[4] = pivot;
    info[5] = m;
    info[6] = kmin;
    info[7] = 0;
done:
    free(canon);
    free(newid);
    free(cnt);
    free(g);
    free(elite);
    free(idx);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Iterated SPVAR (Sec. II.B: ISPVAR): sample, fix, continue on the        */
/* reduced problem; fixes are never undone.  Round r uses seed + r.        */
/*   fixed_mask/fixed_val [n]: cumulative fixes in original indices.       */
/*   round_info [rounds][4]: n_free after the round, cumulative offset,    */
/*     best full-problem energy of the round's sample, variables fixed in  */
/*     the round.  Returns the number of rounds run (>= 0) or an error.    */
/* ---------------------------------------------------------------------- */
int orc_ispvar(const orc_problem *P, const double *betas, int32_t sweeps, int32_t reads,
               uint64_t seed, int32_t rounds, double elite_frac, double threshold, int32_t gauge,
               uint8_t *fixed_mask, int8_t *fixed_val, int64_t *round_info)
{
    int32_t n = P->n, nnz = P->row_ptr[n], rd, i, ran = 0;
    int32_t *rp[2], *cl[2], *jv[2], *hv[2], *orig_cur, *orig_new, *orig_tmp;
    uint8_t *co[2], *fm;
    int8_t *fv, *spins;
    int64_t *E, info[8], offset_total = 0;
    orc_problem cur;
    int rc = ORC_OK, b;
    for (b = 0; b < 2; ++b) {
        rp[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        cl[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        jv[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        hv[b] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        co[b] = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    }
    orig_cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orig_new = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    fm = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    fv = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    spins = (int8_t *)malloc((size_t)reads * (n > 0 ? n : 1));
    E = (int64_t *)malloc(sizeof(int64_t) * (size_t)(reads > 0 ? reads : 1));
    if (!orig_cur || !orig_new || !fm || !fv || !spins || !E) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (b = 0; b < 2; ++b)
        if (!rp[b] || !cl[b] || !jv[b] || !hv[b] || !co[b]) {
            rc = ORC_ENOMEM;
            goto done;
        }
    memcpy(rp[0], P->row_ptr, sizeof(int32_t) * (size_t)(n + 1));
    memcpy(cl[0], P->col, sizeof(int32_t) * (size_t)nnz);
    memcpy(jv[0], P->J, sizeof(int32_t) * (size_t)nnz);
    memcpy(hv[0], P->h, sizeof(int32_t) * (size_t)n);
    memcpy(co[0], P->colour, (size_t)n);
    for (i = 0; i < n; ++i) {
        orig_cur[i] = i;
        fixed_mask[i] = 0;
        fixed_val[i] = 0;
    }
    cur = *P;
    b = 0;
    for (rd = 0; rd < rounds; ++rd) {
        int64_t best = INT64_MAX;
        int32_t r;
        cur.row_ptr = rp[b];
        cur.col = cl[b];
        cur.J = jv[b];
        cur.h = hv[b];
        cur.colour = co[b];
        if (cur.n == 0)
            break;
        rc = orc_sa_sample(&cur, betas, sweeps, seed + (uint64_t)rd, 0, 0, reads, NULL, NULL,
                           spins, E);
        if (rc)
            goto done;
        for (r = 0; r < reads; ++r)
            if (E[r] < best)
                best = E[r];
        rc = orc_persist_fix(&cur, spins, E, reads, elite_frac, threshold, gauge, fm, fv,
                             rp[1 - b], cl[1 - b], jv[1 - b], hv[1 - b], co[1 - b], orig_new, info);
        if (rc)
            goto done;
        for (i = 0; i < cur.n; ++i)
            if (fm[i]) {
                fixed_mask[orig_cur[i]] = 1;
                fixed_val[orig_cur[i]] = fv[i];
            }
        for (i = 0; i < (int32_t)info[0]; ++i)
            orig_new[i] = orig_cur[orig_new[i]];
        orig_tmp = orig_cur;
        orig_cur = orig_new;
        orig_new = orig_tmp;
        round_info[rd * 4 + 0] = info[0];
        round_info[rd * 4 + 2] = best + offset_total;
        offset_total += info[2];
        round_info[rd * 4 + 1] = offset_total;
        round_info[rd * 4 + 3] = info[3];
        cur.n = (int32_t)info[0];
        b = 1 - b;
        ran = rd + 1;
    }
    rc = ran;
done:
    for (b = 0; b < 2; ++b) {
        free(rp[b]);
        free(cl[b]);
        free(jv[b]);
        free(hv[b]);
        free(co[b]);
    }
    free(orig_cur);
    free(orig_new);
    free(fm);
    free(fv);
    free(spins);
    free(E);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Disconnected problems (Sec. II.C special considerations).              */
/* ---------------------------------------------------------------------- */

/* Component of every variable (breadth-first search from the smallest
 * unvisited index); returns the number of components or a negative status. */
int32_t orc_components(const orc_problem *P, int32_t *comp)
{
    int32_t n = P->n, c = 0, i;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue)
        return ORC_ENOMEM;
    for (i = 0; i < n; ++i)
        comp[i] = -1;
    for (i = 0; i < n; ++i) {
        int32_t head = 0, tail = 0;
        if (comp[i] >= 0)
            continue;
        comp[i] = c;
        queue[tail++] = i;
        while (head < tail) {
            int32_t v = queue[head++], k;
            for (k = P->row_ptr[v]; k < P->row_ptr[v + 1]; ++k) {
                int32_t j = P->col[k];
                if (P->J[k] != 0 && comp[j] < 0) {
                    comp[j] = c;
                    queue[tail++] = j;
                }
            }
        }
        ++c;
    }
    free(queue);
    return c;
}

typedef struct {
    int64_t e;
    int32_t row;
} part_key;

static int cmp_part(const void *a, const void *b)
{
    const part_key *x = (const part_key *)a, *y = (const part_key *)b;
    if (x->e != y->e)
        return x->e < y->e ? -1 : 1;
    return (x->row > y->row) - (x->row < y->row);
}

/* Sorted-merge recombination of a sample of R rows.  merged [R][n],
 * merged_E [R]; part_E (optional) [n_comp][R] receives each component's
 * partial energies in its sorted order. */
int orc_merge_sorted(const orc_problem *P, const int32_t *comp, int32_t n_comp, const int8_t *samples,
                     int32_t R, int8_t *merged, int64_t *merged_E, int64_t *part_E)
{
    int32_t n = P->n, r, i, c, k;
    int64_t *pe;
    part_key *keys;
    if (n_comp < 0 || R < 0)
        return ORC_EINVAL;
    pe = (int64_t *)calloc((size_t)(R > 0 ? R : 1) * (size_t)(n_comp > 0 ? n_comp : 1), sizeof(int64_t));
    keys = (part_key *)malloc(sizeof(part_key) * (size_t)(R > 0 ? R : 1));
    if (!pe || !keys) {
        free(pe);
        free(keys);
        return ORC_ENOMEM;
    }
    /* partial energies: every bias and every coupler once, charged to the
     * component of its variables */
    for (r = 0; r < R; ++r) {
        const int8_t *s = samples + (size_t)r * n;
        for (i = 0; i < n; ++i) {
            int64_t e = (int64_t)P->h[i] * s[i];
            for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
                int32_t j = P->col[k];
                if (j > i)
                    e += (int64_t)P->J[k] * s[i] * s[j];
            }
            pe[(size_t)r * n_comp + comp[i]] += e;
        }
    }
    for (k = 0; k < R; ++k)
        merged_E[k] = 0;
    for (c = 0; c < n_comp; ++c) {
        for (r = 0; r < R; ++r) {
            keys[r].e = pe[(size_t)r * n_comp + c];
            keys[r].row = r;
        }
        qsort(keys, (size_t)R, sizeof(part_key), cmp_part);
        for (k = 0; k < R; ++k) {
            const int8_t *src = samples + (size_t)keys[k].row * n;
            merged_E[k] += keys[k].e;
            if (part_E)
                part_E[(size_t)c * R + k] = keys[k].e;
            for (i = 0; i < n; ++i)
                if (comp[i] == c)
                    merged[(size_t)k * n + i] = src[i];
        }
    }
    free(pe);
    free(keys);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Multi-start SPVAR (Algorithm 2).                                        */
/* ---------------------------------------------------------------------- */

int orc_tree_peel(const orc_problem *P, uint8_t *kind, int8_t *value, int32_t *parent, int32_t *round,
                  int32_t *row_ptr_o, int32_t *col_o, int32_t *J_o, int32_t *h_o, uint8_t *colour_o,
                  int32_t *orig_o, int64_t *info);
int orc_tree_expand(int32_t n, const uint8_t *kind, const int8_t *value, const int32_t *parent,
                    const int32_t *round, const int32_t *orig, int32_t n_free, int32_t rounds,
                    const int8_t *reduced, int32_t R, int8_t *full);

/* One reduction of a start's problem: a persistence step (type 1) or a tree
 * peel (type 2), with the problem it leaves. */
typedef struct {
    int32_t type, n_prev, n_next, rounds;
    int64_t offset;
    int32_t *orig;            /* [n_next] -> index in the previous problem */
    int8_t *val;              /* [n_prev] type 1: fixed value or 0; type 2: tree value */
    uint8_t *kind, *mask;     /* [n_prev] type 2: tree kind; type 1: fixed mask */
    int32_t *parent, *round;  /* [n_prev] type 2 */
    int32_t *rp, *cl, *jv, *hv;
    uint8_t *co;
    orc_problem out;
} ms_level;

static int ms_level_alloc(ms_level *L, int32_t n, int32_t nnz)
{
    size_t nn = (size_t)(n > 0 ? n : 1), zz = (size_t)(nnz > 0 ? nnz : 1);
    memset(L, 0, sizeof *L);
    L->orig = (int32_t *)malloc(4 * nn);
    L->val = (int8_t *)malloc(nn);
    L->kind = (uint8_t *)malloc(nn);
    L->mask = (uint8_t *)malloc(nn);
    L->parent = (int32_t *)malloc(4 * nn);
    L->round = (int32_t *)malloc(4 * nn);
    L->rp = (int32_t *)malloc(4 * (nn + 1));
    L->cl = (int32_t *)malloc(4 * zz);
    L->jv = (int32_t *)malloc(4 * zz);
    L->hv = (int32_t *)malloc(4 * nn);
    L->co = (uint8_t *)malloc(nn);
    return (L->orig && L->val && L->kind && L->mask && L->parent && L->round && L->rp && L->cl && L->jv &&
            L->hv && L->co) ? ORC_OK : ORC_ENOMEM;
}

static void ms_level_free(ms_level *L)
{
    free(L->orig); free(L->val); free(L->kind); free(L->mask); free(L->parent); free(L->round);
    free(L->rp); free(L->cl); free(L->jv); free(L->hv); free(L->co);
    memset(L, 0, sizeof *L);
}

static void ms_level_out(ms_level *L, const orc_problem *Q, int32_t n_next)
{
    L->n_prev = Q->n;
    L->n_next = n_next;
    L->out = *Q;
    L->out.n = n_next;
    L->out.row_ptr = L->rp;
    L->out.col = L->cl;
    L->out.J = L->jv;
    L->out.h = L->hv;
    L->out.colour = L->co;
}

/* Persistence (Algorithm 1) on a sample of Q as a level; info as orc_persist_fix. */
static int ms_persist(const orc_problem *Q, const int8_t *S, const int64_t *E, int32_t R, double elite, double thr,
                      int32_t gauge, ms_level *L, int64_t *info)
{
    int rc = orc_persist_fix(Q, S, E, R, elite, thr, gauge, L->mask, L->val, L->rp, L->cl, L->jv, L->hv, L->co,
                             L->orig, info);
    if (rc)
        return rc;
    L->type = 1;
    L->offset = info[2];
    ms_level_out(L, Q, (int32_t)info[0]);
    return ORC_OK;
}

/* Tree peel of Q as a level; info as orc_tree_peel. */
static int ms_tree(const orc_problem *Q, ms_level *L, int64_t *info)
{
    int rc = orc_tree_peel(Q, L->kind, L->val, L->parent, L->round, L->rp, L->cl, L->jv, L->hv, L->co, L->orig,
                           info);
    if (rc)
        return rc;
    L->type = 2;
    L->offset = info[2];
    L->rounds = (int32_t)info[5];
    ms_level_out(L, Q, (int32_t)info[0]);
    return ORC_OK;
}

/* A state of the problem left by levels lv[0..top-1] (of the base problem when
 * top == 0), lifted through the levels in reverse to the base problem.  a and b
 * hold the base size. */
static void ms_lift(const ms_level *const *lv, int32_t top, const int8_t *state, int32_t n_base, int8_t *a,
                    int8_t *b, int8_t *out)
{
    int32_t k, i, u, n_cur = top > 0 ? lv[top - 1]->n_next : n_base;
    int8_t *cur = a, *prev = b, *t;
    memcpy(cur, state, (size_t)n_cur);
    for (k = top - 1; k >= 0; --k) {
        const ms_level *L = lv[k];
        if (L->type == 1) {
            for (i = 0; i < L->n_prev; ++i)
                prev[i] = L->val[i];
            for (u = 0; u < L->n_next; ++u)
                prev[L->orig[u]] = cur[u];
        } else {
            orc_tree_expand(L->n_prev, L->kind, L->val, L->parent, L->round, L->orig, L->n_next, L->rounds, cur,
                            1, prev);
        }
        t = cur;
        cur = prev;
        prev = t;
    }
    memcpy(out, cur, (size_t)n_base);
}

/* One sampling stage: the reads [r0, r0 + R) of a job on Q with `seed`: SA
 * (sampler 0) or SQA over `trotter` slices with the Gamma schedule (sampler 1). */
static int ms_sample(const orc_problem *Q, const orc_ms_params *p, uint64_t seed, int32_t r0, int32_t R,
                     int8_t *spins, int64_t *E)
{
    int32_t *bk;
    int rc;
    if (p->sampler == 0)
        return orc_sa_sample(Q, p->betas, p->sweeps, seed, 0, r0, r0 + R, NULL, NULL, spins, E);
    if (p->sampler != 1 || !p->gammas)
        return ORC_EINVAL;
    bk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R > 0 ? R : 1));
    if (!bk)
        return ORC_ENOMEM;
    rc = orc_sqa_sample(Q, p->betas, p->gammas, p->sweeps, p->trotter, seed, r0, r0 + R, NULL, NULL, spins, E, bk);
    free(bk);
    return rc;
}

/* Sample split of the parameter appendix: zero-bias problems give 40 % of the
 * total to the correlation step and halve the rest between fixing and solving
 * (fixing takes the odd read); otherwise fixing and solving halve it. */
void orc_ms_split(int32_t total, int32_t zero_bias, int32_t *corr, int32_t *fix, int32_t *solve)
{
    int32_t c = zero_bias ? (int32_t)(((int64_t)2 * total) / 5) : 0, rest = total - c;
    *corr = c;
    *fix = (rest + 1) / 2;
    *solve = rest - *fix;
}

/* R99 of a multi-start run (Sec. III.A): p = fraction of starts whose lowest
 * recorded energy reaches e_target; starts for 99 % confidence n99 =
 * ln(0.01) / ln(1 - p), at least one start (so 1 when p >= 0.99), not rounded;
 * R99 = n99 * per_start (the total sample of one start).  p == 0: not
 * measurable, returns -1. */
double orc_r99(const int64_t *start_best, int32_t starts, int64_t e_target, double per_start, double *p_out)
{
    int32_t s, hit = 0;
    double p, n99;
    for (s = 0; s < starts; ++s)
        hit += start_best[s] <= e_target;
    p = starts > 0 ? (double)hit / (double)starts : 0.0;
    if (p_out)
        *p_out = p;
    if (hit == 0)
        return -1.0;
    n99 = hit == starts ? 1.0 : log(0.01) / log(1.0 - p);
    if (n99 < 1.0)
        n99 = 1.0;
    return n99 * per_start;
}

int orc_multistart(const orc_problem *P, const orc_ms_params *p, orc_ms_out *o)
{
    int32_t n = P->n, nnz = P->row_ptr[n], S = p->starts, s, r, i, k;
    int32_t Rc = p->corr_reads, F = p->fixing_reads, Rs = p->solving_reads;
    int32_t Rmax = Rc > F ? Rc : F;
    ms_level pre, lv_own[4];
    const ms_level *lv[5];
    orc_problem base = *P;
    int64_t off_pre = 0, best = INT64_MAX, info[8];
    int8_t *smp = NULL, *mg = NULL, *la = NULL, *lb = NULL, *lifted = NULL;
    int64_t *E = NULL;
    int32_t *map = NULL, *map2 = NULL, *comp = NULL;
    int32_t n_pre_lv = 0, n_base, kinds[4], nst;
    int rc = ORC_OK;
    memset(&pre, 0, sizeof pre);
    memset(lv_own, 0, sizeof lv_own);
    if (S < 1 || F < 1 || Rc < 0 || Rs < 0 || (Rc > 0 && !(p->corr_elite_frac > 0.0)) || p->corr_after < 0 ||
        p->corr_after > 1 || p->preprocess < 0 || p->preprocess > 3)
        return ORC_EINVAL;
    if (Rs > Rmax)
        Rmax = Rs;
    if (n < 1)
        return ORC_EINVAL;
    smp = (int8_t *)malloc((size_t)Rmax * n);
    mg = (int8_t *)malloc((size_t)Rmax * n);
    E = (int64_t *)malloc(sizeof(int64_t) * (size_t)Rmax);
    la = (int8_t *)malloc((size_t)n);
    lb = (int8_t *)malloc((size_t)n);
    lifted = (int8_t *)malloc((size_t)n);
    map = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    map2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!smp || !mg || !E || !la || !lb || !lifted || !map || !map2 || !comp) {
        rc = ORC_ENOMEM;
        goto done;
    }
    /* [Optional] pre-processing of the problem before the loop */
    if (p->preprocess & 1) {
        if ((rc = ms_level_alloc(&pre, n, nnz)) || (rc = ms_tree(P, &pre, info)))
            goto done;
        for (k = 0; k < 8; ++k)
            o->info_pre[k] = info[k];
        base = pre.out;
        off_pre = pre.offset;
        lv[0] = &pre;
        n_pre_lv = 1;
    } else {
        for (k = 0; k < 8; ++k)
            o->info_pre[k] = 0;
        o->info_pre[0] = n;
        o->info_pre[1] = nnz;
    }
    n_base = n;
    for (k = 0; k < 4; ++k)
        if ((rc = ms_level_alloc(&lv_own[k], n, nnz)))
            goto done;
    /* the stages of every start, in order: 0 correlation, 1 SPVAR fixing, 2 tree, 3 solving */
    nst = 0;
    if (Rc > 0 && p->corr_after == 0)
        kinds[nst++] = 0;
    kinds[nst++] = 1;
    if (p->preprocess & 2)
        kinds[nst++] = 2;
    if (Rc > 0 && p->corr_after == 1)
        kinds[nst++] = 0;
    for (s = 0; s < S; ++s) {
        const orc_problem *Q = &base;
        int64_t off = off_pre, sbest = INT64_MAX;
        int32_t depth = n_pre_lv, nlev = 0, k_sample = 0, j;
        int64_t *oinfo = o->info + (size_t)s * 8;
        uint8_t *fm = o->fixed_mask + (size_t)s * n;
        int8_t *fv = o->fixed_val + (size_t)s * n;
        for (i = 0; i < 8; ++i)
            oinfo[i] = 0;
        oinfo[6] = -1;
        for (i = 0; i < n; ++i) {
            fm[i] = 0;
            fv[i] = 0;
        }
        for (i = 0; i < base.n; ++i)
            map[i] = n_pre_lv ? pre.orig[i] : i;
        for (j = 0; j <= nst; ++j) {
            const int32_t kind = j < nst ? kinds[j] : 3;
            int32_t R = kind == 0 ? Rc : kind == 1 ? F : kind == 3 ? Rs : 0;
            int64_t *rec = kind == 0 ? o->corr_E + (size_t)s * Rc
                                     : kind == 1 ? o->fixing_E + (size_t)s * F : o->solving_E + (size_t)s * Rs;
            ms_level *L;
            if (kind == 3 && Rs == 0)
                break;
            if (kind != 2) {
                /* a sample of the current problem, recorded in full-problem units */
                if (Q->n > 0) {
                    if (k_sample == 0)
                        rc = ms_sample(Q, p, p->seed, s * R, R, smp, E);
                    else
                        rc = ms_sample(Q, p, p->seed + 1 + (uint64_t)(k_sample - 1) * S + (uint64_t)s, 0, R, smp,
                                       E);
                    if (rc)
                        goto done;
                    if (kind == 3 && p->merge) {
                        int32_t nc = orc_components(Q, comp);
                        if (nc < 0) {
                            rc = nc;
                            goto done;
                        }
                        if ((rc = orc_merge_sorted(Q, comp, nc, smp, R, mg, E, NULL)))
                            goto done;
                        memcpy(smp, mg, (size_t)R * Q->n);
                        oinfo[5] = nc;
                    }
                } else {
                    for (r = 0; r < R; ++r)
                        E[r] = 0;
                }
                ++k_sample;
                for (r = 0; r < R; ++r) {
                    rec[r] = E[r] + off;
                    if (rec[r] < sbest)
                        sbest = rec[r];
                    if (rec[r] < best) {
                        best = rec[r];
                        ms_lift(lv, depth, smp + (size_t)r * Q->n, n_base, la, lb, lifted);
                        memcpy(o->best_spins, lifted, (size_t)n);
                    }
                }
                if (kind == 3)
                    break;
            }
            if (Q->n == 0)
                continue; /* nothing left to fix or peel */
            L = &lv_own[nlev];
            if (kind == 2) {
                if ((rc = ms_tree(Q, L, info)))
                    goto done;
                oinfo[2] += info[3] + info[4];
            } else {
                const int corr = kind == 0;
                if ((rc = ms_persist(Q, smp, E, R, corr ? p->corr_elite_frac : p->elite_frac,
                                     corr ? p->corr_threshold : p->threshold, corr ? 1 : p->gauge, L, info)))
                    goto done;
                for (i = 0; i < L->n_prev; ++i)
                    if (L->mask[i]) {
                        fm[map[i]] = 1;
                        fv[map[i]] = L->val[i];
                    }
                oinfo[corr ? 0 : 1] += info[3];
                if (corr && info[4] >= 0)
                    oinfo[6] = map[info[4]];
            }
            for (i = 0; i < L->n_next; ++i)
                map2[i] = map[L->orig[i]];
            memcpy(map, map2, sizeof(int32_t) * (size_t)L->n_next);
            off += L->offset;
            lv[depth++] = L;
            ++nlev;
            Q = &L->out;
        }
        oinfo[3] = Q->n;
        oinfo[4] = off;
        o->start_best[s] = sbest;
    }
    *o->best_E = best;
done:
    ms_level_free(&pre);
    for (k = 0; k < 4; ++k)
        ms_level_free(&lv_own[k]);
    free(smp); free(mg); free(E); free(la); free(lb); free(lifted); free(map); free(map2); free(comp);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Tree pre-processing (Sec. II.C).                                        */
/* ---------------------------------------------------------------------- */

/* kind [n]: 0 remaining, 1 fixed, 2 inferred; value [n]: the fixed value, or
 * for an inferred variable the factor f with s = f * s_parent; parent [n];
 * round [n] (-1 for remaining variables); reduced CSR (row_ptr_o [n+1], col_o,
 * J_o, h_o, colour_o), orig_o [n'] (reduced -> original); info [8] = n_free,
 * nnz_free, offset, n_fixed, n_inferred, rounds, 0, n_removed. */
int orc_tree_peel(const orc_problem *P, uint8_t *kind, int8_t *value, int32_t *parent, int32_t *round,
                  int32_t *row_ptr_o, int32_t *col_o, int32_t *J_o, int32_t *h_o, uint8_t *colour_o,
                  int32_t *orig_o, int64_t *info)
{
    int32_t n = P->n, i, k, rd = 0;
    int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *nbk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *peel = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int32_t *newidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t offset = 0, n_fixed = 0, n_inf = 0;
    int32_t nf = 0, nz = 0;
    if (!h || !deg || !nb || !nbk || !peel || !newidx) {
        free(h); free(deg); free(nb); free(nbk); free(peel); free(newidx);
        return ORC_ENOMEM;
    }
    for (i = 0; i < n; ++i) {
        h[i] = P->h[i];
        kind[i] = 0;
        value[i] = 0;
        parent[i] = -1;
        round[i] = -1;
    }
    for (;;) {
        int32_t any = 0;
        /* degrees and the single remaining neighbour of every remaining variable */
        for (i = 0; i < n; ++i) {
            deg[i] = 0;
            nb[i] = -1;
            nbk[i] = -1;
            if (kind[i] != 0)
                continue;
            for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
                if (P->J[k] != 0 && kind[P->col[k]] == 0) {
                    ++deg[i];
                    nb[i] = P->col[k];
                    nbk[i] = k;
                }
        }
        for (i = 0; i < n; ++i) {
            peel[i] = 0;
            if (kind[i] != 0 || deg[i] > 1)
                continue;
            if (deg[i] == 1 && deg[nb[i]] == 1 && nb[i] > i)
                continue; /* an isolated pair: the larger index goes first */
            peel[i] = 1;
            any = 1;
        }
        if (!any)
            break;
        for (i = 0; i < n; ++i) {
            int64_t hi = h[i];
            if (!peel[i])
                continue;
            round[i] = rd;
            if (deg[i] == 0) {
                int8_t s = hi > 0 ? -1 : 1;
                kind[i] = 1;
                value[i] = s;
                offset += hi * s;
                ++n_fixed;
            } else {
                int32_t j = nb[i];
                int64_t Jv = P->J[nbk[i]], aJ = Jv < 0 ? -Jv : Jv, ah = hi < 0 ? -hi : hi;
                parent[i] = j;
                if (aJ <= ah) {
                    int8_t s = hi > 0 ? -1 : 1;
                    kind[i] = 1;
                    value[i] = s;
                    h[j] += Jv * s;
                    offset += hi * s;
                    ++n_fixed;
                } else {
                    int8_t f = Jv > 0 ? -1 : 1;
                    kind[i] = 2;
                    value[i] = f;
                    h[j] += f * hi; /* -sign(J) h */
                    offset -= aJ;
                    ++n_inf;
                }
            }
        }
        ++rd;
    }
    /* reduced problem over the remaining variables, in index order */
    for (i = 0; i < n; ++i)
        newidx[i] = kind[i] == 0 ? nf++ : -1;
    row_ptr_o[0] = 0;
    for (i = 0; i < n; ++i) {
        if (kind[i] != 0)
            continue;
        orig_o[newidx[i]] = i;
        h_o[newidx[i]] = (int32_t)h[i];
        colour_o[newidx[i]] = P->colour[i];
        for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
            if (kind[P->col[k]] == 0) {
                col_o[nz] = newidx[P->col[k]];
                J_o[nz] = P->J[k];
                ++nz;
            }
        row_ptr_o[newidx[i] + 1] = nz;
    }
    info[0] = nf;
    info[1] = nz;
    info[2] = offset;
    info[3] = n_fixed;
    info[4] = n_inf;
    info[5] = rd;
    info[6] = 0;
    info[7] = n - nf; /* removed variables */
    free(h); free(deg); free(nb); free(nbk); free(peel); free(newidx);
    return ORC_OK;
}

/* Completion of reduced states: full [R][n] from reduced [R][n_free]. */
int orc_tree_expand(int32_t n, const uint8_t *kind, const int8_t *value, const int32_t *parent,
                    const int32_t *round, const int32_t *orig, int32_t n_free, int32_t rounds,
                    const int8_t *reduced, int32_t R, int8_t *full)
{
    int32_t r, i, rd;
    for (r = 0; r < R; ++r) {
        int8_t *s = full + (size_t)r * n;
        for (i = 0; i < n_free; ++i)
            s[orig[i]] = reduced[(size_t)r * n_free + i];
        for (rd = rounds - 1; rd >= 0; --rd)
            for (i = 0; i < n; ++i)
                if (round[i] == rd)
                    s[i] = kind[i] == 1 ? value[i] : (int8_t)(value[i] * s[parent[i]]);
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Colour classes by Jones-Plassmann rounds (definition in the header).    */
/* ---------------------------------------------------------------------- */
static int prio_gt(uint32_t pa, int32_t a, uint32_t pb, int32_t b)
{
    return pa > pb || (pa == pb && a > b);
}

int orc_colour_jp(const orc_problem *P, uint64_t seed, uint8_t *colour, int32_t *n_colours, int32_t max_colours)
{
    const int32_t n = P->n;
    int32_t i, k, left = n, used_max = 0;
    uint32_t *prio = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!prio || !col || !next) {
        free(prio); free(col); free(next);
        return ORC_EINVAL;
    }
    for (i = 0; i < n; ++i) {
        prio[i] = philox_word((uint32_t)i, 0u, 0u, 5u << 24, seed, 0);
        col[i] = -1;
    }
    while (left > 0) {
        /* decide on the state at the start of the round */
        for (i = 0; i < n; ++i) {
            next[i] = -1;
            if (col[i] >= 0) continue;
            {
                int top = 1;
                for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k) {
                    const int32_t j = P->col[k];
                    if (col[j] < 0 && prio_gt(prio[j], j, prio[i], i)) {
                        top = 0;
                        break;
                    }
                }
                if (top) {
                    int32_t c = 0, again = 1;
                    while (again) {
                        again = 0;
                        for (k = P->row_ptr[i]; k < P->row_ptr[i + 1]; ++k)
                            if (col[P->col[k]] == c) {
                                ++c;
                                again = 1;
                                break;
                            }
                    }
                    next[i] = c;
                }
            }
        }
        for (i = 0; i < n; ++i)
            if (next[i] >= 0) {
                col[i] = next[i];
                --left;
                if (next[i] + 1 > used_max) used_max = next[i] + 1;
            }
    }
    *n_colours = used_max > 0 ? used_max : 1;
    if (used_max > max_colours) {
        free(prio); free(col); free(next);
        return ORC_ERANGE;
    }
    for (i = 0; i < n; ++i) colour[i] = (uint8_t)col[i];
    free(prio); free(col); free(next);
    return ORC_OK;
}
