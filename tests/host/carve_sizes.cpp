// Host check of the library's workspace carving: the size a dry run of a
// problem's carve reports (base null, which sizes every workspace) must equal
// what the carve takes when it has a base, for every parameter set the
// library accepts; a carve that takes more writes past the block its caller
// sized.  Prints one line per case and exits with the number of mismatches.
#include <cstdio>

#include "fld.h"
#include "fld_engine.h"

using namespace fld;

int main() {
  const int shapes[][3] = {{8, 8, 8}, {32, 32, 32}, {16, 24, 32}, {64, 64, 64},
                           {48, 32, 16}, {128, 4, 6}};
  int bad = 0, cases = 0;
  for (const auto &s : shapes) {
    for (int prec = 0; prec < 2; ++prec) {
      for (int variant = 0; variant < 5; ++variant) {
        fld_params p;
        fld_default_params(&p, 3e10, 1.0);
        p.precision = prec;
        if (variant == 1) p.local_sweeps = 0;
        if (variant == 2) p.smoother = FLD_SMOOTH_JACOBI;
        if (variant == 3) p.nu_pre = p.nu_post = 2;
        if (variant == 4) p.direction_fp64 = 0;
        fld_grid g{};
        g.nx = s[0];
        g.ny = s[1];
        g.nz = s[2];
        g.dx = g.dy = g.dz = 1.0;
        const Hier h = make_hier(g, p);
        Carver dry, real;
        real.base = reinterpret_cast<char *>(1ull << 40);
        ProbMem m1, m2;
        carve_problem(dry, h, p, m1);
        carve_problem(real, h, p, m2);
        const bool ok = dry.off == real.off && align_up(real.off) == problem_bytes(h, p);
        printf("%dx%dx%d prec %d variant %d: dry %zu carved %zu %s\n", s[0], s[1], s[2],
               prec, variant, dry.off, real.off, ok ? "ok" : "MISMATCH");
        bad += !ok;
        ++cases;
      }
    }
  }
  printf("%d cases, %d mismatches\n", cases, bad);
  return bad;
}
