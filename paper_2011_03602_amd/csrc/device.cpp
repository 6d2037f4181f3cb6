// Device identity for keys that must not mix measurements from different
// hardware (the tile tuners' measurement file).
#include "ofl_internal.hpp"

namespace ofl {

std::string device_arch(int device) {
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    return prop.gcnArchName;
}

}  // namespace ofl
