/* Plain C client of libwqa's ABI (host-only context: no GPU needed).  Prints one line per
 * check; the test that builds it compares the printed values with the Python binding. */
#include <stdio.h>
#include <stdlib.h>

#include "wqa.h"

int main(void) {
    wqa_ctx *ctx = NULL;
    if (wqa_abi_version() != WQA_ABI_VERSION) return 10;
    if (wqa_create(&ctx, -1) != WQA_OK) return 11;
    const int64_t n_el[3] = {4, 5, 6};
    if (wqa_set_space(ctx, 3, 3, n_el) != WQA_OK) return 12;
    if (wqa_set_default_rules(ctx) != WQA_OK) return 13;
    int64_t rows = 0, slots = 0, points = 0, dims[3] = {0, 0, 0};
    if (wqa_query(ctx, &rows, &slots, &points, dims) != WQA_OK) return 14;
    printf("rows %lld slots %lld points %lld grid %lld %lld %lld\n", (long long)rows, (long long)slots,
           (long long)points, (long long)dims[0], (long long)dims[1], (long long)dims[2]);
    double x[9 * 4], w[9 * 4];     /* direction 2: n = 6 + 3 functions, 4 nodes each */
    if (wqa_get_rules(ctx, WQA_MASS, 2, x, w) != WQA_OK) return 15;
    double sum = 0.0;
    for (int i = 0; i < 9 * 4; ++i) sum += w[i];
    printf("mass omegas sum %.17g first node %.17g\n", sum, x[0]);
    /* misuse: an assemble call on a host-only context, a bad final mode */
    if (wqa_assemble_mass(ctx, WQA_F32, NULL, NULL, NULL) != WQA_ESTATE) return 16;
    printf("estate: %s\n", wqa_last_error());
    if (wqa_set_final_mode(ctx, (wqa_final)7) != WQA_EINVAL) return 17;
    wqa_destroy(ctx);
    printf("ok\n");
    return 0;
}
