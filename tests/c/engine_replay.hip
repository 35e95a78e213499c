// Host replay of recorded dot-product streams through the library's scalar engine:
// engine_column (any l) and engine_column_l<L> (the form the kernels run) must
// leave the same state, byte for byte, after every column.  Input file: the
// number of cases, then per case a header "name l ncols beta abs_tol sigma_0 ..
// sigma_{l-1}" and ncols lines "c raw_0 .. raw_l" (raw_0 = (z_c, v_{c-l}),
// raw_m = (z_c, z_{c-l+m}); nan where the index is negative).  Prints one line
// per case: status and last_t after the last column fed (columns stop being fed
// once the engine reports a stop) and "identical" or "MISMATCH"; exit code 1 on
// any mismatch.
#include "plcg_device.h"
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
using namespace plcg;

template <int L>
int run_l(DevState &a, DevState &b, const double *raw, int c) {
  engine_column(a, raw, c, nullptr);
  engine_column_l<L>(b, raw, c, nullptr);
  return memcmp(&a, &b, sizeof(DevState));
}

int dispatch(int l, DevState &a, DevState &b, const double *raw, int c) {
  switch (l) {
    case 1: return run_l<1>(a, b, raw, c);
    case 2: return run_l<2>(a, b, raw, c);
    case 3: return run_l<3>(a, b, raw, c);
    case 4: return run_l<4>(a, b, raw, c);
    case 5: return run_l<5>(a, b, raw, c);
    case 6: return run_l<6>(a, b, raw, c);
    case 7: return run_l<7>(a, b, raw, c);
    case 8: return run_l<8>(a, b, raw, c);
  }
  return -1;
}

int main(int argc, char **argv) {
  FILE *f = fopen(argv[1], "r");
  int ncases;
  if (fscanf(f, "%d", &ncases) != 1) return 2;
  int bad = 0;
  for (int cs = 0; cs < ncases; ++cs) {
    char name[128];
    int l, ncols;
    double beta, abs_tol, sig[kLMax] = {0};
    if (fscanf(f, "%127s %d %d %lf %lf", name, &l, &ncols, &beta, &abs_tol) != 5) return 3;
    for (int k = 0; k < l; ++k)
      if (fscanf(f, "%lf", &sig[k]) != 1) return 4;
    DevState a;
    memset(&a, 0, sizeof(a));
    a.l = l;
    for (int k = 0; k < kLMax; ++k) a.sigma[k] = sig[k];
    a.beta = beta;
    a.rref = beta;
    a.abs_tol = abs_tol;
    a.status = kRunning;
    a.last_t = -1;
    gref(a, 0, 0) = 1.0;
    DevState b = a;
    int ran = 0, mism = 0;
    for (int q = 0; q < ncols; ++q) {
      int c;
      double raw[kLMax + 1];
      if (fscanf(f, "%d", &c) != 1) return 5;
      for (int m = 0; m <= l; ++m) {
        char tok[64];
        if (fscanf(f, "%63s", tok) != 1) return 6;
        raw[m] = strtod(tok, nullptr);
      }
      if (a.status != kRunning) continue;
      ++ran;
      if (dispatch(l, a, b, raw, c) != 0) {
        ++mism;
        if (mism < 3) printf("  %s: state differs after column %d\n", name, c);
      }
    }
    printf("%-14s l=%d columns=%d status=%d last_t=%d cols=%d %s\n", name, l, ran, a.status,
           a.last_t, a.cols, mism ? "MISMATCH" : "identical");
    bad += mism != 0;
  }
  return bad ? 1 : 0;
}
