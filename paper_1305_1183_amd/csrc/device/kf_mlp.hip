// kf_mlp.hip -- learned cost model kernels (filled in later).
