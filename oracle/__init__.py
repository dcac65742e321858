"""FP64 CPU oracles, written from the paper and pinned by the tests.

* ``cavi_oracle`` (C and Python): the mixture CAVI sweep;
* ``mlp_oracle``: the warm-start MLP (forward, backward, AdamW);
* ``lmvb_oracle``: the paper's variational Bayes for its linear-mixing model (eqs 16-31);
* ``lmem_oracle``: its EM (eqs 42-47);
* ``gibbs_oracle``: its Gibbs sampler (eqs 32-40), with counter-based draws.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the GPU library never imports, links or calls it.
"""
