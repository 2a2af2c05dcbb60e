// Host-only stand-in for the library's device layer, for the sanitizer build
// of the host C++ (transcription, symbolic analysis, C ABI): no device is
// present, so every device entry answers NO_DEVICE and nothing is allocated.
// Test infrastructure only; the library itself never links this file.
#include <string>
#include <vector>

#include "../../paper_2606_04725_amd/csrc/internal.h"

namespace nmpc {
namespace {
nmpc_status none(std::string& err) {
    err = "no HIP device (sanitizer build)";
    return NMPC_ERR_NO_DEVICE;
}
}  // namespace

bool device_present() { return false; }
nmpc_status device_init(Problem&, std::string& err) { return none(err); }
void device_free(Problem&) {}
void device_invalidate_adjoint(Problem&) {}
nmpc_status device_set_parameters(Problem&, std::string& err) { return none(err); }
nmpc_status device_set_parameters_dev(Problem&, const double*, const double*, const double*, const double*, void*,
                                      std::string& err) { return none(err); }
nmpc_status device_get_solution_dev(const Problem&, double*, double*, double*, double*, double*, double*, double*,
                                    void*, std::string& err) { return none(err); }
nmpc_status device_adjoint_dev(Problem&, const double*, const double*, double*, double*, double*, double*, void*,
                               std::string& err) { return none(err); }
nmpc_status device_solve(Problem&, int, const nmpc_options&, nmpc_result&, std::string& err) { return none(err); }
nmpc_status device_closed_loop(Problem&, int, const double*, const double*, double*, double*, int,
                               const nmpc_options&, void*, int*, int*, std::string& err) { return none(err); }
nmpc_status device_get_iterate(const Problem&, double*, double*, double*, double*, double*, double*,
                               std::string& err) { return none(err); }
nmpc_status device_get_first_stage(const Problem&, double*, double*, std::string& err) { return none(err); }
nmpc_status device_set_iterate(Problem&, const double*, const double*, const double*, const double*, const double*,
                               const double*, std::string& err) { return none(err); }
nmpc_status device_eval(Problem&, const double*, const double*, const double*, double*, double*, double*, double*,
                        double*, double*, std::string& err) { return none(err); }
nmpc_status device_factor(Problem&, const double*, double, int32_t*, double*, std::string& err) { return none(err); }
nmpc_status device_linear_solve(Problem&, const double*, double*, std::string& err) { return none(err); }
nmpc_status device_assemble(Problem&, double, double*, double*, std::string& err) { return none(err); }
nmpc_status device_adjoint(Problem&, const double*, double, double*, double*, double*, double*, std::string& err) {
    return none(err);
}
nmpc_status device_jacobian_u1_x0(Problem&, double*, std::string& err) { return none(err); }
size_t noalloc_scratch_bytes(const Problem&) { return 0; }
nmpc_status device_jacobian_u1_x0_noalloc(Problem&, double*, void*, std::string& err) { return none(err); }
nmpc_status device_autotune(Problem&, int, int*, std::string& err) { return none(err); }
nmpc_status batch_create(const std::vector<Problem*>&, Batch*&, std::string& err) { return none(err); }
void batch_free(Batch*) {}
nmpc_status batch_solve(Batch&, int, const nmpc_options&, nmpc_result*, std::string& err) { return none(err); }
}  // namespace nmpc
