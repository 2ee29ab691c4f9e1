"""Host planner: the paper's cost model, Greedy / RandomGreedy paths and the
simulated-annealing partition refinement."""
from . import cost
from .greedy import greedy_pairs, random_greedy_pairs
from .plan import Plan, contiguous_partition, plan_from_partition, build_part, assemble_tree
from .sa import SAConfig, simulated_annealing
from .slicing import choose_slices, contract_sliced, sliced_problem
