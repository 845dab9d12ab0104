// std_sort_context.cpp -- GNU std::sort on one host thread (TEST INFRASTRUCTURE).
//
// The paper measures its method against the C++ standard library's sort on one
// pinned core (Sec. IV-A).  The benchmark times this on the same bounded
// sample as the oracle and prints it beside the oracle's time, as context
// only; nothing here is part of the library or checks its output.
#include <algorithm>
#include <cstdint>

extern "C" {

void context_std_sort_i32(int32_t *a, int64_t n) { std::sort(a, a + n); }

void context_std_sort_f64(double *a, int64_t n) { std::sort(a, a + n); }

}  // extern "C"
