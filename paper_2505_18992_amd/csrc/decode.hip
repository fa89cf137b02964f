// decode.hip -- anchor -> neural-Gaussian decode (placeholder until the
// decoder kernels land).
#include "internal.h"

extern "C" {

int vpgs_decode_forward(vpgs_ctx*, const vpgs_anchors*, const vpgs_mlp*, const float*, const vpgs_gauss_buffers*,
                        void*) {
  return VPGS_EUNSUPPORTED;
}

int vpgs_decode_backward(vpgs_ctx*, const vpgs_anchors*, const vpgs_mlp*, const float*, const vpgs_gauss_grads*,
                         float*, float*, float*, const vpgs_mlp_grads*, void*) {
  return VPGS_EUNSUPPORTED;
}

}
