// Live timing of one selected kernel of the hot path with HIP events.
//
// When a kernel id is selected (ot_kprof_select), every launch of that kernel
// is made through hipExtLaunchKernelGGL with a start / stop event pair, which
// the runtime stamps at the dispatch's own start and end on the stream it
// runs on, and its algorithmic HBM bytes (the minimum traffic the launch must
// move: every operand read once, every result written once) are added up on
// the host.  Event pairs come from a pool that is drained (synchronised and
// summed) when full and on read-out.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <utility>
#include <vector>

namespace otbb {
namespace kprof {

struct Prof {
    std::mutex mu;
    int sel = 0;                                         // OT_KPROF_* id, 0 = off
    int width = 0;                                       // element bytes to count, 0 = any
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<double> pend;                            // bytes of pending launches
    size_t used = 0;
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};

// event pair for one launch; both null when the kernel is not selected
struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
};

Prof &prof();
void drain(Prof &P);          // caller holds P.mu
Ev take_slot(double bytes);   // books one launch of the selected kernel

// elem: bytes per element of the launch's floating-point operands
inline Ev take(int id, int elem, double bytes) {
    const Prof &P = prof();
    if (id == 0 || P.sel != id || (P.width != 0 && P.width != elem)) return Ev{};
    return take_slot(bytes);
}

}  // namespace kprof
}  // namespace otbb
