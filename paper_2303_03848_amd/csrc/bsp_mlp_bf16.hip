// Network forward pass on the matrix cores (bfloat16 inputs, float32 accumulation).
#include "bsp_common.hpp"

namespace bsp {

struct NetInput;
int launch_mlp_bf16(const pinn_net& net, long n, const NetInput& in, float* out32, double* out64,
                    double scale, hipStream_t stream) {
    (void)net; (void)n; (void)in; (void)out32; (void)out64; (void)scale; (void)stream;
    set_error("bfloat16 network path not built");
    return BS_ERR_ARG;
}

}  // namespace bsp
