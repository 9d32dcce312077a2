/* Host-only use of the C ABI from plain C (no GPU needed): validation,
 * stability limit, sizes, error codes and messages, teardown. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mp.h"

static void binary_params(mp_params* p) {
    memset(p, 0, sizeof *p);
    p->precision = MP_FP64;
    p->potential = MP_WELL;
    p->eps = 4.0;
    p->tau = 1.0;
    p->gamma[0][1] = p->gamma[1][0] = 1.0;
    p->A[0][0] = p->A[1][0] = 1.0;
    p->B[0][0] = -0.4;
    p->B[1][0] = -1.6;
    p->D[1][0] = 1.0;
    p->dt = 1e-3; /* validated with the rest; the limit itself does not depend on it */
}

int main(void) {
    mp_grid g;
    memset(&g, 0, sizeof g);
    g.dim = 2;
    g.n[0] = 64;
    g.n[1] = 48;
    g.n[2] = 1;
    g.dx = 1.0;
    mp_params p;
    binary_params(&p);

    const double lim = mp_dt_limit(&g, 2, 2, &p);
    /* dx^2/(2d) min(tau / (2 gamma (N-1)/N), chi / (D chi)) = 0.25 min(1, 1) */
    if (fabs(lim - 0.25) > 1e-15) {
        printf("dt limit %.17g\n", lim);
        return 1;
    }
    p.dt = 0.2 * lim;
    mp_state* st = NULL;
    int rc = mp_create(&g, 2, 2, &p, &st);
    if (rc != MP_OK || !st) {
        printf("create %d: %s\n", rc, mp_last_error());
        return 2;
    }
    if (mp_state_bytes(st) != (size_t)(64 * 48 * 3 * 8) || mp_workspace_bytes(st) == 0) return 3;
    int which = -1;
    int64_t step = -1;
    if (mp_current(st, &which, &step) != MP_OK || which != 0 || step != 0) return 4;
    /* stepping before mp_bind is refused, with a message */
    if (mp_step(st, 1, NULL) != MP_E_UNBOUND || strlen(mp_last_error()) == 0) return 5;
    /* so is stepping with the diagnostics; a NULL output is refused first */
    mp_diag d;
    if (mp_step_diag(st, 1, &d, NULL) != MP_E_UNBOUND) return 13;
    if (mp_step_diag(st, 1, NULL, NULL) != MP_E_NULLPTR) return 14;
    /* the anti-trapping switch: off by default, on (both forms) and off again, 3 refused */
    int on = -1;
    if (mp_get_antitrapping(st, &on) != MP_OK || on != 0) return 9;
    if (mp_set_antitrapping(st, 2) != MP_OK || mp_get_antitrapping(st, &on) != MP_OK || on != 2) return 10;
    if (mp_set_antitrapping(st, 1) != MP_OK || mp_get_antitrapping(st, &on) != MP_OK || on != 1) return 10;
    if (mp_set_antitrapping(st, 3) != MP_E_PARAM) return 11;
    if (mp_set_antitrapping(st, 0) != MP_OK || mp_get_antitrapping(st, &on) != MP_OK || on != 0) return 12;
    mp_destroy(st);

    /* too large a time step, and an unsupported phase count */
    p.dt = 2.0 * lim;
    st = NULL;
    if (mp_create(&g, 2, 2, &p, &st) != MP_E_UNSTABLE || st) return 6;
    p.dt = 0.2 * lim;
    if (mp_create(&g, 4, 2, &p, &st) != MP_E_PARAM || st) return 7;
    if (mp_create(NULL, 2, 2, &p, &st) != MP_E_NULLPTR) return 8;
    printf("ok\n");
    return 0;
}
