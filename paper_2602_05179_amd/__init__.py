"""MI355X-native scenario-batched split evaluator (CVRP with stochastic demand).

The evaluation runs in the HIP library libsplit_eval.so (C ABI in
include/split_eval.h); `paper_2602_05179_amd.binding` is its Python binding
and `paper_2602_05179_amd.workloads` draws seeded synthetic inputs.
"""
