// Kernel launches that report their own status.
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace xg {

// Enqueues kernel<<<grid, block, lds, stream>>>(args...) through
// hipLaunchKernel and returns the status of this launch alone.  (Reading
// hipGetLastError after a launch would also return an error that an unrelated
// earlier HIP call left behind on the same host thread.)  The arguments are
// converted to the kernel's parameter types before their addresses are taken.
template <typename... P, typename... A>
inline hipError_t launch(void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                         A &&...args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  std::tuple<std::decay_t<P>...> held(std::forward<A>(args)...);
  return std::apply(
      [&](auto &...v) {
        void *argv[] = {static_cast<void *>(&v)...};
        return hipLaunchKernel(reinterpret_cast<const void *>(kernel), grid, block, argv, lds, stream);
      },
      held);
}

}  // namespace xg
