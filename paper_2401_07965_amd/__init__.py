"""Population annealing (Ebert, Gessert, Janke, Weigel, "Optimized population
Monte Carlo") on MI355X: a HIP library behind a small C ABI (include/pa.h)
and its Python binding (``pa``)."""
