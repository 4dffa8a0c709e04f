#include <stdexcept>

#include "tree.hpp"

namespace nce {
void build_tree(const std::vector<double>&, int64_t, double, const PatchTables&, double, Tree&) {
    throw std::runtime_error("tree far field not available in this build");
}
void upload_tree(const Tree&, hipStream_t, DeviceTree&) {}
void free_tree(DeviceTree&) {}
template <class T>
hipError_t tree_far(hipStream_t, const DeviceTree&, int, const double*, const T*, const T*) {
    return hipErrorNotSupported;
}
template <class T>
hipError_t tree_near(hipStream_t, const DeviceTree&, int, const double*, const T*, const T*, const T*, T*) {
    return hipErrorNotSupported;
}
template <class T>
hipError_t tree_interp(hipStream_t, const DeviceTree&, const double*, const T*, T*) {
    return hipErrorNotSupported;
}
template hipError_t tree_far<double>(hipStream_t, const DeviceTree&, int, const double*, const double*, const double*);
template hipError_t tree_far<float>(hipStream_t, const DeviceTree&, int, const double*, const float*, const float*);
template hipError_t tree_near<double>(hipStream_t, const DeviceTree&, int, const double*, const double*, const double*,
                                      const double*, double*);
template hipError_t tree_near<float>(hipStream_t, const DeviceTree&, int, const double*, const float*, const float*,
                                     const float*, float*);
template hipError_t tree_interp<double>(hipStream_t, const DeviceTree&, const double*, const double*, double*);
template hipError_t tree_interp<float>(hipStream_t, const DeviceTree&, const double*, const float*, float*);
}  // namespace nce
