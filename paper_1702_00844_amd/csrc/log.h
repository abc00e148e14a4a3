// The library's event log (host code only).
#pragma once

namespace xc {

// One line to the log named by XC_LOG (unset or "0": no log; "1" or "stderr":
// standard error; anything else: a file appended to), for events that happen
// once per plan, stream or tuning run, never per correlation.
void log_line(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

}  // namespace xc
