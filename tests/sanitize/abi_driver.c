/*
 * Drives the host-side validation of the library's C ABI (include/fastfca.h)
 * with invalid arguments, for a build whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Every call here must be rejected on the host, before any GPU work, so the
 * driver runs on a machine without a GPU. Exit status 0 when every call
 * returned the expected error and no sanitizer fired.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fastfca.h"

static int failures = 0;

static void expect(const char *what, int got, int want)
{
    if (got != want) {
        printf("%s: got %d, expected %d\n", what, got, want);
        ++failures;
    }
}

int main(void)
{
    fastfca_ctx *ctx = (fastfca_ctx *)0x1;
    const void *fake = (const void *)(uintptr_t)4096;   /* never dereferenced: rejected first */
    /* shapes and NULL input of the context constructors */
    expect("init F=0", fastfca_init(&ctx, fake, 0, 10, 2, 3, NULL, NULL, NULL, 0, NULL), FASTFCA_E_ARG);
    expect("init ctx cleared", ctx == NULL, 1);
    expect("init M=1", fastfca_init(&ctx, fake, 4, 10, 1, 3, NULL, NULL, NULL, 0, NULL), FASTFCA_E_ARG);
    expect("init N=1", fastfca_init(&ctx, fake, 4, 10, 2, 1, NULL, NULL, NULL, 0, NULL), FASTFCA_E_ARG);
    expect("init T<M", fastfca_init(&ctx, fake, 4, 1, 2, 3, NULL, NULL, NULL, 0, NULL), FASTFCA_E_ARG);
    expect("init M=9", fastfca_init(&ctx, fake, 4, 100, 9, 3, NULL, NULL, NULL, 0, NULL), FASTFCA_E_UNSUPPORTED);
    expect("init x=NULL", fastfca_init(&ctx, NULL, 4, 100, 2, 3, NULL, NULL, NULL, 0, NULL), FASTFCA_E_ARG);
    expect("error text", strlen(fastfca_last_error(NULL)) > 0, 1);
    expect("init_blocks T%B", fastfca_init_blocks(&ctx, fake, 4, 10, 2, 3, 3, NULL, NULL, NULL, 0, NULL),
           FASTFCA_E_ARG);
    expect("init_batch B=0", fastfca_init_batch(&ctx, 0, NULL, 0, NULL), FASTFCA_E_ARG);
    /* calls on a NULL context */
    expect("em_step NULL", fastfca_em_step(NULL, 1), FASTFCA_E_ARG);
    expect("sync NULL", fastfca_sync(NULL), FASTFCA_E_ARG);
    expect("loglik NULL", fastfca_loglik(NULL, 0, NULL, NULL), FASTFCA_E_ARG);
    expect("mwf NULL", fastfca_mwf(NULL, 0, NULL), FASTFCA_E_ARG);
    expect("get_params NULL", fastfca_get_params(NULL, 0, NULL, NULL, NULL), FASTFCA_E_ARG);
    expect("set_params NULL", fastfca_set_params(NULL, 0, NULL, NULL, NULL), FASTFCA_E_ARG);
    expect("shape NULL", fastfca_shape(NULL, 0, NULL, NULL, NULL, NULL), FASTFCA_E_ARG);
    expect("num_problems NULL", fastfca_num_problems(NULL), FASTFCA_E_ARG);
    expect("set_config NULL", fastfca_set_config(NULL, 256, 4), FASTFCA_E_ARG);
    expect("set_algorithm NULL", fastfca_set_algorithm(NULL, 1), FASTFCA_E_ARG);
    expect("set_ll_alarm NULL", fastfca_set_ll_alarm(NULL, 1e-3), FASTFCA_E_ARG);
    expect("set_tail_split NULL", fastfca_set_tail_split(NULL, 4), FASTFCA_E_ARG);
    expect("warmstart NULL", fastfca_warmstart(NULL, 0, NULL, NULL), FASTFCA_E_ARG);
    expect("warmstart_race NULL", fastfca_warmstart_race(NULL, 0, NULL, 10, NULL), FASTFCA_E_ARG);
    fastfca_destroy(NULL);
    /* the allocation-free entry point: argument and size checks */
    void *p = (void *)(uintptr_t)4096;
    expect("noalloc status NULL", fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 5, NULL, NULL, NULL),
           FASTFCA_E_ARG);
    expect("noalloc n_iter 0", fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 0, p, NULL, NULL), FASTFCA_E_ARG);
    expect("noalloc M=9", fastfca_fit_noalloc(p, 9, 100, 9, 3, p, p, p, 5, p, NULL, NULL), FASTFCA_E_UNSUPPORTED);
    expect("noalloc too big", fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 200000, p, NULL, NULL), FASTFCA_E_ARG);
    expect("noalloc error text", strstr(fastfca_last_error(NULL), "scratch") != NULL, 1);
    /* network entry points */
    expect("pack NULL", fastfca_net_pack_weights(NULL, 16, 4, 2, 5, 16, 0, NULL, NULL), FASTFCA_E_ARG);
    expect("conv mode", fastfca_net_conv_fwd(fake, 1, 2, 8, fake, 16, 5, NULL, 4, (float *)p, 9, NULL, NULL, NULL),
           FASTFCA_E_ARG);
    expect("pit N=5", fastfca_net_pit_loss(fake, fake, fake, fake, 1, 5, 2, 8, 0.5f, (float *)p, NULL, NULL, NULL,
                                           NULL),
           FASTFCA_E_ARG);
    expect("adamw step 0", fastfca_net_adamw((float *)p, fake, (float *)p, (float *)p, 4, 1e-3f, 0.9f, 0.999f,
                                             1e-8f, 0.0f, 0, 1.0f, NULL),
           FASTFCA_E_ARG);
    expect("features M=5", fastfca_ws_features(fake, 4, 8, 5, 1e-8f, p, (float *)p, NULL), FASTFCA_E_ARG);
    expect("net error text", strlen(fastfca_net_last_error()) > 0, 1);
    printf(failures ? "abi driver: %d failures\n" : "abi driver: ok\n", failures);
    return failures != 0;
}
