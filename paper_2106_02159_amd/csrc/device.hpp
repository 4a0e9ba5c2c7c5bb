// device.hpp -- the HIP device of the calling thread, for host code built
// without the HIP headers (the server's set-up threads).
#pragma once

namespace ns {
int current_device();         // hipGetDevice; 0 if it fails
void use_device(int device);  // hipSetDevice
}  // namespace ns
