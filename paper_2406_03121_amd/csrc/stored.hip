// mess_jk(MESS_JK_STORED): unique integral blocks computed once per
// (basis, precision, threshold) and streamed on every later call.
#include "class_ops.hpp"
#include "mess_internal.hpp"

namespace mess {

struct StoredEri {
    int prec = MESS_FP64;
    double tau = 0.0;
};

void free_stored(mess_basis *B) {
    for (auto &kv : B->stored) delete kv.second;
    B->stored.clear();
}

int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s) {
    (void)B; (void)D; (void)Gj; (void)Gk; (void)prec; (void)tau; (void)s;
    set_error("mess_jk: MESS_JK_STORED is not built yet");
    return MESS_E_UNSUPPORTED;
}

}  // namespace mess
