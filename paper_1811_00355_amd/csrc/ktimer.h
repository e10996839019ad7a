// Per-kernel event timing hooks (see ktimer.hip).
#pragma once
#include "dd_internal.h"

bool ktimer_enabled(const char* tag);
void ktimer_begin(const char* tag, hipStream_t st);
void ktimer_end(const char* tag, hipStream_t st, double bytes, double flops);
void ktimer_suspend(bool on);   // while on, no launch of this thread is timed

// Algorithmic work model of this thread's launches: every instrumented launch
// adds its bytes and flops (timed or not); a replayed graph adds what its
// capture recorded.  dd_solve reports the totals of one call.
void ktimer_account(double bytes, double flops);
void ktimer_model(double* bytes, double* flops);
void ktimer_model_set(double bytes, double flops);

// Launch `launch` (a kernel launch statement) bracketed by timing events when
// the kernel name `tag` is being timed; `bytes` / `flops` are the launch's
// algorithmic traffic and arithmetic.
#define DD_TIMED(tag, st, bytes, flops, launch)             \
  do {                                                      \
    const bool _on = ktimer_enabled(tag);                   \
    const double _b = (bytes), _f = (flops);                \
    if (_on) ktimer_begin(tag, st);                         \
    launch;                                                 \
    if (_on) ktimer_end(tag, st, _b, _f);                   \
    ktimer_account(_b, _f);                                 \
  } while (0)
