// host_internal.h -- host helpers shared by the library's translation units.
#ifndef ASTERX_HOST_INTERNAL_H
#define ASTERX_HOST_INTERNAL_H

namespace axh {
// Records msg as the calling thread's last error (asterx_last_error) and returns code.
int set_error(int code, const char* msg);
}  // namespace axh

#endif
