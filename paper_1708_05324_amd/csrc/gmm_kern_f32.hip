// FP32 (complex64 field) instantiation of the propagation kernels.
#include "gmm_launch_impl.hpp"
template struct gmm::Launch<float>;
