// Structure tables of the CPTP generator (host side, plain C++).
#pragma once
#include <vector>

namespace gst {

// y [D][D] (by a, b), zr / zi [D][D][D] (by j, a, b) for n qubits (D = 4^n); see
// gst_param_tables.cpp.
void param_tables(int n, std::vector<double>* y, std::vector<double>* zr, std::vector<double>* zi);

}  // namespace gst
