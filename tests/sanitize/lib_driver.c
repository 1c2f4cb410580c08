/* Host-side driver for the sanitizer build of libgws (AddressSanitizer + UndefinedBehavior-
 * Sanitizer on the host code only; no device is needed): every host-only entry point --
 * problem validation, workspace sizing for each path, status text, version, and the
 * argument checks of the device entry points -- with valid and invalid arguments.  Prints OK
 * and exits 0 when every call returned what include/gws.h documents. */
#include <stdio.h>
#include <string.h>
#include "gws.h"
int main(void) {
    int bad = 0;
    gws_problem p; memset(&p, 0, sizeof(p));
    p.nx = 1920; p.ny = 1080; p.pitch_x = p.pitch_y = 8e-6; p.n_lambda = 3;
    p.lambdas[0] = 638e-9; p.lambdas[1] = 520e-9; p.lambdas[2] = 450e-9;
    size_t b = 0;
    bad |= gws_check_problem(&p) != GWS_OK;
    bad |= gws_workspace_size(NULL, &p, 100000, &b) != GWS_OK || b == 0;
    bad |= gws_workspace_size_tilted(NULL, &p, 100000, &b) != GWS_OK || b == 0;
    int64_t off[4] = {0, 10, 1000, 100000};
    bad |= gws_workspace_size_batched(NULL, &p, 3, off, &b) != GWS_OK || b == 0;
    p.blend = GWS_BLEND_EXACT;
    bad |= gws_workspace_size(NULL, &p, 1000, &b) != GWS_OK || b == 0;
    bad |= gws_workspace_size_batched(NULL, &p, 3, off, &b) != GWS_OK || b == 0;
    p.blend = GWS_BLEND_OIT; p.xform = GWS_XFORM_DFT_BF16X3;
    bad |= gws_workspace_size(NULL, &p, 1000, &b) != GWS_OK || b == 0;
    bad |= gws_dft_workspace_size(NULL, 3840, 2160, 3, GWS_XFORM_DFT_BF16X3, &b) != GWS_OK || b == 0;
    bad |= gws_focal_stack_workspace_size(NULL, &p, 8, 0, &b) != GWS_OK || b == 0;
    bad |= gws_dpac_workspace_size(3) == 0 || gws_l2_workspace_size() == 0;
    /* rejected shapes and arguments */
    p.nx = 1921; bad |= gws_check_problem(&p) == GWS_OK; p.nx = 1920;
    p.n_lambda = 5; bad |= gws_check_problem(&p) == GWS_OK; p.n_lambda = 3;
    p.pitch_x = -1.0; bad |= gws_check_problem(&p) == GWS_OK; p.pitch_x = 8e-6;
    p.eps_support = 1.0; bad |= gws_check_problem(&p) == GWS_OK; p.eps_support = 0.0;
    bad |= gws_workspace_size(NULL, &p, -5, &b) == GWS_OK;
    bad |= gws_workspace_size_tilted(NULL, &p, -5, &b) == GWS_OK;
    int64_t badoff[3] = {0, 50, 20};
    bad |= gws_workspace_size_batched(NULL, &p, 2, badoff, &b) == GWS_OK;
    bad |= gws_dft_workspace_size(NULL, 7, 9, 1, 0, &b) == GWS_OK;
    for (int s = -12; s <= 0; ++s) bad |= gws_status_string((gws_status)s) == NULL;   /* unknown codes included */
    bad |= gws_abi_version() != GWS_ABI_VERSION;
    gws_ctx *ctx = NULL;
    gws_status st = gws_create(&ctx, 0);
    if (st == GWS_OK) { gws_destroy(ctx); printf("device present\n"); }
    bad |= gws_last_error(NULL) == NULL;
    bad |= gws_forward(NULL, &p, NULL, NULL, NULL, 0, NULL) == GWS_OK;
    bad |= gws_forward_tilted(NULL, &p, NULL, NULL, NULL, 0, NULL) == GWS_OK;
    bad |= gws_backward(NULL, &p, NULL, NULL, NULL, NULL, 0, NULL) == GWS_OK;
    bad |= gws_backward_tilted(NULL, &p, NULL, NULL, NULL, NULL, 0, NULL) == GWS_OK;
    bad |= gws_destroy(NULL) != GWS_OK;
    printf("%s\n", bad ? "FAIL" : "OK");
    return bad;
}
