// Live timing of one selected kernel of the hot path with HIP events.
//
// When a kernel id is selected (ot_kprof_select), every launch of that kernel
// is bracketed by a pair of events recorded on the stream it is launched on,
// and its algorithmic HBM bytes (the minimum traffic the launch must move:
// every operand read once, every result written once) are added up on the
// host.  Event pairs come from a pool that is drained (synchronised and
// summed) when full and on read-out, so the overhead per launch is two
// event records.
#pragma once

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
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<double> pend;                            // bytes of pending launches
    size_t used = 0;
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};

Prof &prof();
void drain(Prof &P);          // caller holds P.mu
void begin(hipStream_t s);
void end(hipStream_t s, double bytes);

inline bool on(int id) { return id != 0 && prof().sel == id; }

// RAII bracket around one launch
struct Scope {
    bool active;
    hipStream_t s;
    double bytes;
    Scope(int id, hipStream_t s_, double b) : active(on(id)), s(s_), bytes(b) {
        if (active) begin(s);
    }
    ~Scope() {
        if (!active) return;
        try {
            end(s, bytes);
        } catch (...) {          // a failed record must not escape a destructor
        }
    }
};

}  // namespace kprof
}  // namespace otbb
