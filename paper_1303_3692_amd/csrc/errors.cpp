// Error codes and the thread-local last-error message.
#include "internal.h"

namespace samatch {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace samatch

extern "C" const char *sa_strerror(int code) {
    switch (code) {
        case SA_OK: return "ok";
        case SA_PENDING: return "pending";
        case SA_EINVAL: return "invalid argument";
        case SA_EALPHABET: return "reference byte outside ACGT";
        case SA_ETOOBIG: return "size beyond the supported maximum";
        case SA_ENOMEM: return "out of host memory";
        case SA_EDEVICE: return "HIP device error";
        case SA_ENOSPC: return "request can never fit in device memory";
        case SA_ECANCELED: return "cancelled";
        case SA_EIO: return "file input/output error";
        case SA_EFORMAT: return "bad index file";
        case SA_ENOTFOUND: return "unknown ticket";
        default: return "unknown error code";
    }
}

extern "C" const char *sa_last_error(void) { return samatch::g_last_error.c_str(); }
