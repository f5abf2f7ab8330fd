// GCIN kernels (added with the learned predictor)
