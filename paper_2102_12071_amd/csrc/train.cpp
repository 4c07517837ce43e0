// Training step driver for the high-frequency smoothing loss.
#include "internal.hpp"
#include "launch.hpp"

using namespace mg;

extern "C" mg_status mg_train_step(mg_net net, const mg_train_batch *b, const mg_train_opts *o, float *loss,
                                   float *grad)
{
    clear_error();
    (void)b; (void)o; (void)loss; (void)grad;
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    return set_error(MG_ERR_STATE, "training is not available in this build");
}
