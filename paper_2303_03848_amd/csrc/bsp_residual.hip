// PINN loss and gradient.
#include "bsp_common.hpp"

extern "C" size_t pinn_residual_workspace_size(const pinn_net* net, int n_f, int n_e, int n_b) {
    (void)net; (void)n_f; (void)n_e; (void)n_b;
    return 0;
}

extern "C" int pinn_residual_fwd_bwd(const pinn_net* net, const bs_params* prm, int n_f,
                                     const float* X_f, int n_e, const float* X_e, int n_b,
                                     const float* X_b, float* loss3, float* grad, void* ws,
                                     size_t ws_bytes, void* stream) {
    (void)net; (void)prm; (void)n_f; (void)X_f; (void)n_e; (void)X_e; (void)n_b; (void)X_b;
    (void)loss3; (void)grad; (void)ws; (void)ws_bytes; (void)stream;
    bsp::set_error("not built");
    return BS_ERR_ARG;
}
