"""Repeated ensemble inference for profiling: 65,536 electrode queries (the
surrogate-in-the-loop sweep's distribution) through the 4-net ensemble, 11
calls of sur_infer_route with the committed weights.  --layered runs the
per-layer products (one k_gemm per layer and net) instead of the fused
kernel.

    rocprofv3 --kernel-trace --stats -- python3 -m paper_2207_06908_amd.sur_profile [--layered]
"""
import os
import sys


def main(calls: int = 11, queries: int = 65536, layered: bool = False):
    import torch
    from . import scenarios as S
    from . import surrogate as U
    cases = S.draw_cases(queries, seed=5, widen=0.1)
    X = torch.from_numpy(U.features(cases)).cuda()
    sur = U.Surrogate(n_nets=4, max_rows=queries)
    sur.load(os.path.join(os.path.dirname(U.__file__), "data", "surrogate_weights.npz"))
    if layered:
        sur.ens.set_kernel(0)
    for _ in range(calls):
        sur.ens.infer_route(X, U.FAST_THRESHOLD)
    torch.cuda.synchronize()
    print(f"{calls} {'layered' if layered else 'fused'} inference calls of {queries} queries done", flush=True)


if __name__ == "__main__":
    main(layered="--layered" in sys.argv[1:])
