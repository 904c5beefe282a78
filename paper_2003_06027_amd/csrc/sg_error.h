// sg_error.h -- error reporting shared by the host-side sources of libseisgrad.
#pragma once

namespace sg {

// Records a printf-style message for last_error() and returns `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

} // namespace sg
