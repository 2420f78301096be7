// Error plumbing of the C ABI (every entry point catches, records a
// thread-local message and returns a status) and small device-memory helpers.
#pragma once

#include <new>
#include <string>
#include <vector>

#include "ssamg_impl.h"

namespace ssamg {

void set_last_error(const std::string &msg);

template <typename T>
T *dev_alloc(size_t n) {
  if (n == 0) n = 1;
  void *p = nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(SSAMG_ERR_ALLOC, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return (T *)p;
}

template <typename T>
void dev_upload(T *&dst, const std::vector<T> &src) {
  if (dst) (void)hipFree(dst);
  dst = dev_alloc<T>(src.size());
  if (!src.empty())
    SSAMG_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace ssamg

#define API_BEGIN try {
#define API_END                                                  \
  }                                                              \
  catch (const ::ssamg::Error &e) {                              \
    ::ssamg::set_last_error(e.what());                           \
    return e.code;                                               \
  }                                                              \
  catch (const std::bad_alloc &) {                               \
    ::ssamg::set_last_error("host allocation failed");           \
    return SSAMG_ERR_ALLOC;                                      \
  }                                                              \
  catch (const std::exception &e) {                              \
    ::ssamg::set_last_error(e.what());                           \
    return SSAMG_ERR_ARG;                                        \
  }                                                              \
  ::ssamg::set_last_error("");                                   \
  return SSAMG_OK;
