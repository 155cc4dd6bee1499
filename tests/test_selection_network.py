"""The comparator network that keeps the five nearest of the nine lattice
candidates (Sec. 2, runtime lookup: the K = 5 nearest of up to nine
neighbours) must leave the five smallest keys of any input in positions
0..4, in order.  By the 0-1 principle it is enough to check every input of
zeros and ones; the network is read from the device header."""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1903_03837_amd", "csrc", "sf_search.hpp")


def network(name="kSel5of9"):
    src = open(HDR).read()
    body = re.search(name + r"Net\[" + name + r"\]\[2\] = \{(.*?)\};", src, re.S).group(1)
    pairs = [(int(a), int(b)) for a, b in re.findall(r"\{(\d+),\s*(\d+)\}", body)]
    count = int(re.search(r"constexpr int " + name + r" = (\d+);", src).group(1))
    assert len(pairs) == count
    return pairs


def apply(net, v):
    v = list(v)
    for a, b in net:
        if v[b] < v[a]:
            v[a], v[b] = v[b], v[a]
    return v


def test_network_keeps_five_smallest_on_all_zero_one_inputs():
    net = network()
    assert all(0 <= a < b < 9 for a, b in net)
    for bits in range(1 << 9):
        v = [(bits >> i) & 1 for i in range(9)]
        assert apply(net, v)[:5] == sorted(v)[:5], bits


def test_network_on_random_distinct_keys():
    net = network()
    rng = np.random.default_rng(5)
    for _ in range(2000):
        v = list(rng.permutation(9))
        assert apply(net, v)[:5] == [0, 1, 2, 3, 4]


def test_pruning_is_tight():
    """every comparator is needed: dropping any one breaks the property"""
    net = network()
    for i in range(len(net)):
        t = net[:i] + net[i + 1:]
        bad = any(apply(t, [(b >> k) & 1 for k in range(9)])[:5] != sorted((b >> k) & 1 for k in range(9))[:5]
                  for b in range(1 << 9))
        assert bad, i


def test_four_of_eight_keeps_four_smallest_in_order():
    """The network used when the centre is known to be the nearest candidate:
    the four smallest of the other eight keys, in order, for every input of
    zeros and ones (0-1 principle) and for random distinct keys; every
    comparator is needed."""
    net = network("kSel4of8")
    assert all(0 <= a < b < 8 for a, b in net)
    for bits in range(1 << 8):
        v = [(bits >> i) & 1 for i in range(8)]
        assert apply(net, v)[:4] == sorted(v)[:4], bits
    rng = np.random.default_rng(6)
    for _ in range(2000):
        assert apply(net, list(rng.permutation(8)))[:4] == [0, 1, 2, 3]
    for i in range(len(net)):
        t = net[:i] + net[i + 1:]
        assert any(apply(t, [(b >> k) & 1 for k in range(8)])[:4] != sorted((b >> k) & 1 for k in range(8))[:4]
                   for b in range(1 << 8)), i
