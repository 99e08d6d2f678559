// Host-only probe of the launch cost model of the sweeps (no kernel, no
// device call): for each nx ny nz triple on the command line it prints the
// z chunk of the thesis sweep, the z chunk of the 14-row FP32 sweep, and
// whether the FP32 correction sweep takes its 10-row tiles.
#include <cstdio>
#include "pt_internal.h"
int main(int argc, char** argv) {
    for (int a = 1; a + 2 < argc; a += 3) {
        ptk::Geom g{};
        g.nx = atoi(argv[a]); g.ny = atoi(argv[a + 1]); g.nz = atoi(argv[a + 2]);
        g.P = ((g.nx + 1 + 31) / 32) * 32; g.S = g.P * (g.ny + 1);
        printf("%d %d %d %d %d %d\n", g.nx, g.ny, g.nz, ptk::choose_kz(g, ptk::BX, ptk::BY),
               ptk::choose_kz(g, ptk::BX, ptk::BY_CORR32), (int)ptk::corr32_short(g));
    }
    return 0;
}
