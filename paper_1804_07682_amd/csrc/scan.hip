// Batched chain with the smearing on the matrix cores (filled in below).
#include "gna_internal.h"

namespace gna {

bool scan_supported(const gna_plan* p) {
  (void)p;
  return false;
}

size_t scan_dense_bytes(const gna_plan* p) {
  (void)p;
  return 0;
}

int build_scan_tables(gna_plan* p, hipStream_t s) {
  (void)p;
  (void)s;
  return GNA_OK;
}

int launch_scan(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                double* pred, hipStream_t s) {
  (void)p;
  (void)params;
  (void)B;
  (void)chi2;
  (void)grad;
  (void)pred;
  (void)s;
  return fail(GNA_E_UNSUPPORTED, "MFMA scan kernel not built");
}

}  // namespace gna
