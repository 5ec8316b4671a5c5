// Host-side helpers shared by the single-graph and the batched C calls.
#pragma once

#include "kernels.hpp"

namespace csc {

hipStream_t as_stream(void* s);
csc_status check_graph(const csc_graph* g);
csc_status check_ws(void* ws, size_t ws_bytes, size_t need);
void jackson_lowpass(double lc, int p, double* a);
double count_from_moments(double lambda, int p, const double* mom);
void apply_tuning(StepArgs& sa);
size_t filter_bytes(const Layout& L);
size_t count_bytes(const Layout& L, int p);
size_t interp_bytes(const Layout& L);
int use_hip_graphs();
hipStream_t capture_stream();

}  // namespace csc
