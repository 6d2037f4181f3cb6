// Helpers that keep C++ exceptions from crossing the C interface.
#pragma once

#include <new>
#include <string>

#include "ofl_internal.hpp"

namespace ofl {

void set_last_error(const std::string &msg);

// Run f(); map any exception to a status code and record its message.
// A device error on a handle whose device state exists makes it unusable.
template <class F>
int guarded(bool *broken, F &&f) {
    try {
        f();
        return OFL_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        if (e.code == OFL_EDEVICE && broken)
            *broken = true;
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("out of host memory");
        return OFL_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(std::string("internal error: ") + e.what());
        return OFL_EINVAL;
    } catch (...) {
        set_last_error("unknown internal error");
        return OFL_EINVAL;
    }
}

}  // namespace ofl
