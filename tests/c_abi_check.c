/* A C program against include/fdwave.h and libfdwave.so with no Python and no torch:
 * it calls the host-only entry points (stencil weights, stability limit, workspace
 * sizes, argument validation) and prints what it found, one "key value" pair per
 * line.  Compiled and run by test_abi.py; needs no GPU. */
#include <stdio.h>
#include <string.h>

#include "fdwave.h"

int main(void)
{
    double w[13];
    if (fd_weights(4, w) != FD_OK) return 1;
    printf("w4 %.17g %.17g %.17g %.17g %.17g\n", w[0], w[1], w[2], w[3], w[4]);
    printf("dtmax3_r4 %.17g\n", fd_dt_max(3, 4, 10.0, 4500.0));

    fd_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = 3;
    g.n[0] = 512;
    g.n[1] = 512;
    g.n[2] = 512;
    size_t field = 0, ws = 0;
    if (fd_field_bytes(&g, 4, FD_F32, &field) != FD_OK) return 2;
    if (fd_workspace_bytes(&g, 4, FD_F32, 1, 16384, &ws) != FD_OK) return 3;
    printf("field_bytes %zu\nworkspace_bytes %zu\n", field, ws);

    /* invalid radius and a 2-D grid with nz != 1 are refused with a message */
    int st = fd_weights(0, w);
    printf("bad_radius %d %s\n", st, fd_last_error()[0] ? "msg" : "nomsg");
    g.ndim = 2;
    st = fd_field_bytes(&g, 4, FD_F32, &field);
    printf("bad_grid %d %s\n", st, fd_last_error()[0] ? "msg" : "nomsg");
    return 0;
}
