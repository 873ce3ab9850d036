/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * library's host code (test infrastructure): calls the entry points that need
 * no GPU -- status strings, the scratch and workspace size queries, the
 * validation of portfolio descriptions (good ones, and bad ones that must be
 * rejected with the documented status), and argument checks that fail before
 * any device work -- so the sanitizers watch the host runtime's parsing and
 * layout arithmetic.  Exit status 0 = every check held.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ara.h"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

int main(void)
{
    for (int s = 1; s >= -12; --s) CHECK(ara_status_string(s) != NULL);
    size_t b = 0;
    CHECK(ara_run_scratch_size(1000000, &b) == ARA_OK && b >= 4000000);
    CHECK(ara_run_scratch_size(-1, &b) == ARA_E_INVALID_ARG);
    CHECK(ara_pml_tvar_scratch_size(12345, &b) == ARA_OK && b > 0);
    CHECK(ara_ep_curve_scratch_size(12345, ARA_F64, &b) == ARA_OK && b > 0);
    CHECK(ara_ep_curve_scratch_size(12345, 7, &b) == ARA_E_INVALID_ARG);
    CHECK(ara_batch_scratch_size(64, 1000000, &b) == ARA_OK && b > 0);
    CHECK(ara_batch_scratch_size(0, 10, &b) == ARA_E_INVALID_ARG);

    /* a portfolio of 3 layers with 1, 4 and 0 ELTs over a 1000-event catalogue */
    enum { NR = 50 };
    int32_t ev[NR];
    float mean[NR], si[NR], sc[NR], mx[NR];
    for (int r = 0; r < NR; ++r) {
        ev[r] = r * 19;
        mean[r] = 1e5f * (float)(r + 1);
        si[r] = 0.5f * mean[r];
        sc[r] = r % 2 ? 0.1f * mean[r] : 0.0f;
        mx[r] = 4.0f * mean[r];
    }
    ara_elt_desc elts[5];
    for (int e = 0; e < 5; ++e) {
        elts[e].elt_id = (uint32_t)(10 + e);
        elts[e].n_rows = NR - 7 * e;
        elts[e].event_ids = ev;
        elts[e].mean = mean;
        elts[e].sigma_i = si;
        elts[e].sigma_c = e == 3 ? NULL : sc;
        elts[e].max_loss = mx;
        elts[e].retention = 1e5;
        elts[e].limit = e == 2 ? INFINITY : 5e6;
        elts[e].share = 0.5 + 0.1 * e;
    }
    ara_layer_desc layers[3];
    memset(layers, 0, sizeof layers);
    layers[0].n_elts = 1; layers[0].elts = elts;
    layers[1].n_elts = 4; layers[1].elts = elts + 1;
    layers[2].n_elts = 0; layers[2].elts = NULL;
    for (int l = 0; l < 3; ++l) {
        layers[l].occ_retention = 1e6;
        layers[l].occ_limit = l == 1 ? INFINITY : 2e7;
        layers[l].agg_retention = 5e6;
        layers[l].agg_limit = 1e8;
        layers[l].program_id = (uint32_t)l;
    }
    ara_portfolio_desc pf = {3, layers, 150106326ull, 1, ARA_KEYING_OCCURRENCE};
    size_t ws = 0, ws_pu = 0;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_OK && ws > 0 && ws % 256 == 0);
    pf.su_enabled = 0;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws_pu) == ARA_OK && ws_pu > 0);
    pf.su_enabled = 1;
    pf.keying = 5;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_INVALID_ARG);
    pf.keying = ARA_KEYING_PAPER;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_OK);
    CHECK(ara_portfolio_workspace_size(&pf, 0, &ws) == ARA_E_INVALID_ARG);
    elts[2].share = 1.5;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_BAD_ELT_ROW);
    elts[2].share = 1.0;
    elts[3].retention = -1.0;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_BAD_ELT_ROW);
    elts[3].retention = 0.0;
    layers[1].agg_retention = INFINITY;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_BAD_ELT_ROW);
    layers[1].agg_retention = 0.0;
    elts[4].n_rows = -3;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_INVALID_ARG);
    elts[4].n_rows = 5;
    elts[4].event_ids = NULL;
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_INVALID_ARG);
    layers[2].n_elts = 3;                 /* ELTs but no list */
    CHECK(ara_portfolio_workspace_size(&pf, 1000, &ws) == ARA_E_INVALID_ARG);
    CHECK(ara_portfolio_workspace_size(NULL, 1000, &ws) == ARA_E_INVALID_ARG);

    /* calls that fail on their arguments before touching a device */
    CHECK(ara_run(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == ARA_E_INVALID_ARG);
    CHECK(ara_pml_tvar(NULL, NULL, 0, 0, NULL, 0, NULL, NULL, NULL, 0, NULL) == ARA_E_INVALID_ARG);
    CHECK(ara_load_yet(NULL, 0, 0, NULL, NULL, NULL, NULL, NULL) == ARA_E_INVALID_ARG);
    CHECK(ara_sync_status(NULL, NULL) == ARA_E_INVALID_ARG);
    CHECK(ara_server_create(0, 0, 0, NULL, NULL, NULL, NULL) != ARA_OK);
    ara_destroy(NULL);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host sanitizer driver: all checks held\n");
    return 0;
}
