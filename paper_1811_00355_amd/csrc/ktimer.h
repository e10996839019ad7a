// Per-kernel event timing hooks (see ktimer.hip).
#pragma once
#include "dd_internal.h"

bool ktimer_enabled(const char* tag);
void ktimer_begin(const char* tag, hipStream_t st);
void ktimer_end(const char* tag, hipStream_t st, double bytes, double flops);
void ktimer_suspend(bool on);   // while on, no launch of this thread is timed

// Launch `launch` (a kernel launch statement) bracketed by timing events when
// the kernel name `tag` is being timed; `bytes` / `flops` are the launch's
// algorithmic traffic and arithmetic.
#define DD_TIMED(tag, st, bytes, flops, launch)             \
  do {                                                      \
    const bool _on = ktimer_enabled(tag);                   \
    if (_on) ktimer_begin(tag, st);                         \
    launch;                                                 \
    if (_on) ktimer_end(tag, st, (bytes), (flops));         \
  } while (0)
