// Collocation tables (host only); see tables.cpp.
#pragma once

namespace isdc {
// Nodes tau (M), cumulative matrix Q (M x M, row-major), node-to-node
// matrix S (M x M) and the whole-step weights b (M) for ISDC_NODES_*; any
// output may be NULL.  Returns false for an invalid (kind, M).
bool tables(int kind, int M, double* tau, double* Q, double* S, double* b = nullptr);
}  // namespace isdc
