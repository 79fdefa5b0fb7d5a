// Host build of the library's per-node arithmetic, for CPU tests that compare
// it with the oracle's dense matrices and with finite differences.
#include <hip/hip_runtime.h>

#include "../../paper_1106_0785_amd/csrc/lbm_dual.h"
#include "../../paper_1106_0785_amd/csrc/lbm_node.h"

using namespace lbm;

extern "C" {
void host_moments(const double* f, double* m) { moments_from_f(f, m); }
void host_f_from_moments(const double* m, double* f) { f_from_moments(m, f); }
void host_mt(const double* nu, double* out) { mt_apply(nu, out); }
void host_minvt(const double* lam, double* mu) { minvt_apply(lam, mu); }
void host_feq(int version, const double* c, double* q) {
  if (version == 2)
    equilibrium_moments<2, double>(c[0], c[1], c[2], c[3], q);
  else if (version == 3)
    equilibrium_moments<3, double>(c[0], c[1], c[2], c[3], q);
  else
    equilibrium_moments<1, double>(c[0], c[1], c[2], c[3], q);
}
// d q / d c_a (16 values) by dual numbers
void host_feq_dir(int version, const double* c, int a, double* dq) {
  Dual x[4];
  for (int k = 0; k < 4; ++k) x[k] = Dual(c[k], k == a ? 1.0 : 0.0);
  Dual q[16];
  if (version == 2)
    equilibrium_moments<2, Dual>(x[0], x[1], x[2], x[3], q);
  else if (version == 3)
    equilibrium_moments<3, Dual>(x[0], x[1], x[2], x[3], q);
  else
    equilibrium_moments<1, Dual>(x[0], x[1], x[2], x[3], q);
  for (int k = 0; k < 16; ++k) dq[k] = q[k].d;
}
}
