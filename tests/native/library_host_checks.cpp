// Host-side checks of libspvar built without device code (hipcc --cuda-host-only) under
// AddressSanitizer and UndefinedBehaviorSanitizer: the acceptance-table arithmetic against
// the oracle's independent implementation over a grid of (beta, unit, scale, digit, d),
// the digit and row-length rules, the multi-start sample split and R99, and the argument
// checks of the entry points that run before any device call.  Exit status 0 when every
// check holds.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "spvar.h"

namespace spv {
uint32_t threshold_word(double beta, int64_t unit, int scale_log2, int digit, uint32_t d);
int digits_for(int64_t x_bound);
int table_row_len(int64_t x_bound);
int swap_digits(double dbeta, int scale_log2);
}  // namespace spv

extern "C" {
uint32_t orc_threshold(double beta, int64_t unit, int32_t scale_log2, int32_t digit, uint32_t d);
int32_t orc_swap_digits(double dbeta, int32_t scale_log2);
void orc_ms_split(int32_t total, int32_t zero_bias, int32_t *corr, int32_t *fix, int32_t *solve);
double orc_r99(const int64_t *start_best, int32_t starts, int64_t e_target, double per_start, double *p_out);
}

static int failures = 0;
#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

int main() {
    // acceptance tables: the library's host builder and the oracle's agree word for word
    const double betas[] = {0.0, 1e-4, 0.003, 0.1, 0.37, 1.0, 2.5, 5.0, 40.0};
    for (double beta : betas)
        for (int64_t unit : {1, 2})
            for (int scale : {0, 3, 10, 20})
                for (int digit = 0; digit < 3; ++digit)
                    for (uint32_t d = 0; d < 512; d += 7)
                        CHECK(spv::threshold_word(beta, unit, scale, digit, d) ==
                              orc_threshold(beta, unit, scale, digit, d));
    for (double db : {1e-3, 0.05, 0.2, 1.0})
        for (int scale : {0, 10})
            CHECK(spv::swap_digits(db, scale) == orc_swap_digits(db, scale));
    // digits and row lengths of the base-512 acceptance test
    CHECK(spv::digits_for(0) == 1 && spv::digits_for(511) == 1 && spv::digits_for(512) == 2);
    CHECK(spv::digits_for(512 * 512 - 1) == 2 && spv::digits_for(512 * 512) == 3);
    CHECK(spv::table_row_len(255) == 256 && spv::table_row_len(511) == 512 && spv::table_row_len(512) == 514);
    // multi-start split and R99 against the oracle
    for (int32_t total = 0; total < 400; total += 3)
        for (int32_t zb = 0; zb < 2; ++zb) {
            int32_t a[3], b[3];
            spv_multistart_split(total, zb, &a[0], &a[1], &a[2]);
            orc_ms_split(total, zb, &b[0], &b[1], &b[2]);
            CHECK(a[0] == b[0] && a[1] == b[1] && a[2] == b[2]);
        }
    const int64_t sb[6] = {-10, -12, -12, -11, -12, -10};
    for (int64_t target : {-13, -12, -11, -10}) {
        double p1 = -1, p2 = -2;
        CHECK(spv_r99(sb, 6, target, 500.0, &p1) == orc_r99(sb, 6, target, 500.0, &p2) && p1 == p2);
    }
    CHECK(spv_r99(sb, 6, -12, 500.0, nullptr) > 500.0);
    // argument checks before any device call
    CHECK(spv_version() != nullptr);
    CHECK(spv_last_error(nullptr) != nullptr);
    CHECK(spv_ctx_create(0, nullptr) == SPV_EINVAL);
    spv_ctx_destroy(nullptr);
    spv_problem P{};
    CHECK(spv_problem_check(nullptr, &P, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_sample(nullptr, &P, nullptr, 0, 0, 0, 0, nullptr, nullptr, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_persist_fix(nullptr, &P, nullptr, nullptr, 1, 0.1, 1.0, 0, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_persist_fix_noalloc(nullptr, &P, nullptr, nullptr, 1, 0.1, 1.0, 0, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_multistart(nullptr, &P, nullptr, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_server_create(nullptr, nullptr, nullptr) == SPV_EINVAL);
    CHECK(spv_debug_lds_shadow(nullptr, nullptr, 0) == SPV_EINVAL);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("library host checks: all passed\n");
    return 0;
}
