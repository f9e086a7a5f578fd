// C entry for the CPU test of the generator structure tables (host code only).
#include <string.h>

#include "gst_param_tables.h"

extern "C" void probe_param_tables(int n, double* y, double* zr, double* zi) {
  std::vector<double> a, b, c;
  gst::param_tables(n, &a, &b, &c);
  memcpy(y, a.data(), a.size() * sizeof(double));
  memcpy(zr, b.data(), b.size() * sizeof(double));
  memcpy(zi, c.data(), c.size() * sizeof(double));
}
