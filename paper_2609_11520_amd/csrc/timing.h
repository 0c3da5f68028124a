// Per-kernel timing scopes (see timing.hip).
#pragma once
#include <cstring>

#include "common.h"

namespace fio {
bool timing_on();

class TimingScope {
public:
    TimingScope(const char *name, hipStream_t s);
    ~TimingScope();
    TimingScope(const TimingScope &) = delete;
    TimingScope &operator=(const TimingScope &) = delete;

private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool active_ = false;
};
}  // namespace fio

#define FIO_TIMED(name, stream) ::fio::TimingScope fio_timing_scope_##__LINE__(name, stream)
