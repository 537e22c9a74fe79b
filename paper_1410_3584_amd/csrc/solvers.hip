// Ground-state and dynamics solvers (filled in below the potential path).
#include "nlf_internal.h"

using namespace nlf;

extern "C" {

int nlf_ground_state(nlf_plan* p, const nlf_phys* phys, const nlf_gf_opts* gf, const void* psi0,
                     void* psi, nlf_gs_stats* stats) {
    clear_error();
    (void)p; (void)phys; (void)gf; (void)psi0; (void)psi; (void)stats;
    return set_error(NLF_EUNSUPPORTED, "ground state solver not built yet");
}

int nlf_evolve(nlf_plan* p, const nlf_phys* phys, const nlf_ts_opts* ts, void* psi, double* diag) {
    clear_error();
    (void)p; (void)phys; (void)ts; (void)psi; (void)diag;
    return set_error(NLF_EUNSUPPORTED, "dynamics solver not built yet");
}

}  // extern "C"
